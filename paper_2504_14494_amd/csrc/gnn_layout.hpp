// Parameter-blob offsets and buffer layouts of the GNN-corrected collision.
#pragma once

#include <cstddef>
#include <cstdint>

namespace gnn {

constexpr int HID = 64;            // hidden width
constexpr int NFEAT = 12;          // node features
constexpr int NOUT = 10;           // head outputs: z_0 -> tau_adj, z_1..9 -> delta f
constexpr int EDGE_IN = 2 * HID + 2;
constexpr int NODE_IN = 2 * HID;
constexpr int MAX_ROUNDS = 4;

// Offsets (in floats) of every tensor of the FP32 blob.
struct BlobLayout {
  size_t W1, b1, W2, b2;
  size_t We[MAX_ROUNDS], be[MAX_ROUNDS], Wn[MAX_ROUNDS], bn[MAX_ROUNDS];
  size_t Wh, bh, nparam, mu, sigma, sdelta, total;
};

inline BlobLayout blob_layout(int R) {
  BlobLayout L{};
  size_t o = 0;
  L.W1 = o; o += (size_t)HID * NFEAT;
  L.b1 = o; o += HID;
  L.W2 = o; o += (size_t)HID * HID;
  L.b2 = o; o += HID;
  for (int r = 0; r < R; ++r) {
    L.We[r] = o; o += (size_t)HID * EDGE_IN;
    L.be[r] = o; o += HID;
    L.Wn[r] = o; o += (size_t)HID * NODE_IN;
    L.bn[r] = o; o += HID;
  }
  L.Wh = o; o += (size_t)NOUT * HID;
  L.bh = o; o += NOUT;
  L.nparam = o;
  L.mu = o; o += NFEAT;
  L.sigma = o; o += NFEAT;
  L.sdelta = o; o += 1;
  L.total = o;
  return L;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Activations kept by gnn_forward for gnn_backward, per node:
//   x   [16]  BF16 normalised features (12 used, 4 zero)
//   e1  [64]  BF16 first encoder layer
//   h_r [64]  BF16 node states r = 0..R
//   a_r [64]  BF16 summed messages r = 1..R
//   z   [10]  FP32 head outputs (stored with stride 12)
struct SavedLayout {
  size_t x, e1, h, agg, z, total;
  size_t nodes;
};

inline SavedLayout saved_layout(long long nodes, int R) {
  SavedLayout S{};
  size_t n = (size_t)nodes, o = 0;
  S.nodes = n;
  S.x = o; o += align256(n * 16 * 2);
  S.e1 = o; o += align256(n * HID * 2);
  S.h = o; o += align256(n * HID * 2) * (size_t)(R + 1);
  S.agg = o; o += align256(n * HID * 2) * (size_t)(R > 0 ? R : 1);
  S.z = o; o += align256(n * 12 * 4);
  S.total = o;
  return S;
}

inline size_t saved_bytes(int batch, int nx, int ny, int R) {
  return saved_layout((long long)batch * nx * ny, R).total;
}

// Upper bound on the workgroups of a GNN launch (grids are clamped to it);
// sizes the per-workgroup partial sums.
constexpr int kMaxGnnBlocks = 2048;

// Control words of a step (gate decision and arrival counts, work counters).
constexpr int kCtrlWords = 512;

// Bytes of the packed weight fragments (see gnn_common.hpp); generous bound
// that holds for every n_rounds <= MAX_ROUNDS.
constexpr size_t kPackBytes = 512 * 1024;

// Scratch of one forward pass: packed weights, two BF16 node-state buffers
// (ping-pong), per-workgroup mass and flag partials of the corrected
// collision (fixed point, see gnn_common.hpp) and of the fallback step
// (FP64), and a few control words.
struct ForwardScratch {
  size_t pack, hA, hB, pmass, pflag, pmass2, ctrl, total;
};

constexpr ForwardScratch forward_scratch(long long nodes) {
  ForwardScratch F{};
  size_t n = (size_t)nodes, o = 0;
  F.pack = o; o += kPackBytes;
  F.hA = o; o += align256(n * HID * 2);
  F.hB = o; o += align256(n * HID * 2);
  F.pmass = o; o += align256(kMaxGnnBlocks * 16);  // 16-byte fixed-point partials
  F.pflag = o; o += align256(kMaxGnnBlocks * sizeof(unsigned));
  F.pmass2 = o; o += align256(kMaxGnnBlocks * sizeof(double));
  F.ctrl = o; o += kCtrlWords * 4;
  F.total = o;
  return F;
}

inline size_t forward_workspace_bytes(int batch, int nx, int ny, int R) {
  (void)R;
  return forward_scratch((long long)batch * nx * ny).total;
}

// Scratch of the fused per-node step: packed weights, per-workgroup partials
// of the corrected collision and of the fallback step, control words.
struct SimpleScratch {
  size_t pack, pmass, pflag, pmass2, ctrl, total;
};

inline SimpleScratch simple_scratch() {
  SimpleScratch S{};
  size_t o = 0;
  S.pack = o; o += kPackBytes;
  S.pmass = o; o += align256(kMaxGnnBlocks * 16);  // 16-byte fixed-point partials
  S.pflag = o; o += align256(kMaxGnnBlocks * sizeof(unsigned));
  S.pmass2 = o; o += align256(kMaxGnnBlocks * sizeof(double));
  S.ctrl = o; o += kCtrlWords * 4;
  S.total = o;
  return S;
}

inline size_t step_workspace_bytes(int nx, int ny, int R) {
  return forward_workspace_bytes(1, nx, ny, R);
}

// Backward scratch: packed weights, two FP32 node-gradient buffers
// (ping-pong over the rounds), FP32 gradients of the summed messages, BF16
// per-edge gradients of the edge-layer pre-activations [N][8][64], and one
// FP32 partial parameter gradient per wave of the fixed backward grid.
constexpr int kBwdBlocks = 256;
constexpr int kBwdWaves = kBwdBlocks * 4;
struct BackwardScratch {
  size_t pack, dhA, dhB, dagg, dq, part, total;
};

inline BackwardScratch backward_scratch(long long nodes, int R) {
  BackwardScratch B{};
  size_t n = (size_t)nodes, o = 0;
  size_t np = blob_layout(R).nparam;
  B.pack = o; o += kPackBytes;
  B.dhA = o; o += align256(n * HID * 4);
  B.dhB = o; o += align256(n * HID * 4);
  B.dagg = o; o += align256(n * HID * 4);
  B.dq = o; o += align256(n * 8 * HID * 2);
  B.part = o; o += align256((size_t)kBwdWaves * np * 4);
  B.total = o;
  return B;
}

inline size_t backward_workspace_bytes(int batch, int nx, int ny, int R) {
  return backward_scratch((long long)batch * nx * ny, R).total;
}

}  // namespace gnn
