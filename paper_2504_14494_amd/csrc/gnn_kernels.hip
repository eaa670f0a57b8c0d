// GNN-corrected collision (Eq. 3) on gfx950: weight packing, the node
// encoder, message-passing rounds with the head, projection and corrected
// collision fused into the last round, and the device-side fallback gate.
//
// Network (per node; sizes of the 2048^2 inference workload):
//   x  = (g_0..g_8, rho - 1, u_x, u_y), normalised (x - mu) / sigma      12
//   h0 = GELU(W2 GELU(W1 x + b1) + b2)                          12 -> 64 -> 64
//   round r: m_d = GELU(We [h_n; h_{n+e_d}; e_d] + be) for the 8 neighbours,
//            a = sum_d m_d,  h' = GELU(Wn [h_n; a] + bn)       130 -> 64, 128 -> 64
//   z  = Wh h_R + bh                                                  64 -> 10
//   tau_adj = 1/2 + sigmoid(z_0),  delta f = s_delta P z_{1..9}
//   f*_i = f_i - (f_i - f_i^eq) / (tau tau_adj) + delta f_i                (Eq. 3)
// P is the orthogonal projector onto the null space of the mass and momentum
// moments: with M = [1; e_x; e_y], M M^T = diag(9, 6, 6), so
// (P v)_i = v_i - m0/9 - e_ix mx/6 - e_iy my/6 for the moments (m0, mx, my)
// of v.
//
// The edge layer is split exactly, We [h_n; h_j; e_d] = Wa h_n + Wb h_j +
// Wc e_d: the receiver part Wa h_n + be is formed once per node and seeds the
// accumulator of each of the 8 edges, which then add Wc e_d and Wb h_j with
// MFMA.  All dense layers are BF16 x BF16 -> FP32 MFMA (16x16x32); GELU,
// the message sum and everything after the head run in FP32 on the VALU.
#include <cstdio>
#include <mutex>

#include "channel_common.hpp"
#include "gnn_common.hpp"
#include "lbm_common.hpp"

namespace gnn {

using lbm::cx;
using lbm::cy;

// ------------------------------------------------------------ packing ---

// One thread per (fragment, lane): 8 BF16 A-operand values (or, for bias
// fragments, 4 FP32 accumulator-layout values).  See gnn_common.hpp for the
// fragment conventions.  The index functions give the blob position of a
// value, or -1 for the zero padding, so that a thread can issue all of its
// loads before it waits for any.

// Where the 8 values of one lane of fragment f come from: value j sits at
// base + stride * g(j), with g(j) = frag_channel(s, q, j) (kind 0), 8 q + j
// while below lim (kind 1), or j for q == 0 and j < 2 (kind 2, the two
// edge-direction columns); kind 3 is padding only.  The fragment's kind is
// decoded once per thread: the layout tables are kernel arguments, and
// walking them for each value made the packing a chain of dependent scalar
// loads.
struct FragSrc {
  long long base;
  int stride, kind, s, lim;
};

__host__ __device__ inline FragSrc frag_src(const BlobLayout &L, const FragLayout &F, int R,
                                            int f, int m) {
  FragSrc o{0, 1, 3, 0, 0};
  if (f >= F.W1 && f < F.W1 + 4) {
    o = FragSrc{(long long)(L.W1 + (size_t)(16 * (f - F.W1) + m) * NFEAT), 1, 1, 0, NFEAT};
  } else if (f >= F.W2 && f < F.W2 + 8) {
    const int t = (f - F.W2) >> 1, s = (f - F.W2) & 1;
    o = FragSrc{(long long)(L.W2 + (size_t)(16 * t + m) * HID), 1, 0, s, 0};
  } else if (f >= F.WH && f < F.WH + 2) {
    if (m < NOUT) o = FragSrc{(long long)(L.Wh + (size_t)m * HID), 1, 0, f - F.WH, 0};
  } else if (f >= F.W2T && f < F.W2T + 8) {  // rows: e1 channels, k: h0 channels
    const int t = (f - F.W2T) >> 1, s = (f - F.W2T) & 1;
    o = FragSrc{(long long)(L.W2 + 16 * t + m), HID, 0, s, 0};
  } else if (f >= F.WHT && f < F.WHT + 4) {  // rows: h_R channels, k: head outputs
    o = FragSrc{(long long)(L.Wh + 16 * (f - F.WHT) + m), HID, 1, 0, NOUT};
  } else {
    for (int r = 0; r < R; ++r) {
      const long long We = (long long)L.We[r], Wn = (long long)L.Wn[r];
      if (f >= F.WA[r] && f < F.WA[r] + 8) {
        const int t = (f - F.WA[r]) >> 1, s = (f - F.WA[r]) & 1;
        o = FragSrc{We + (long long)(16 * t + m) * EDGE_IN, 1, 0, s, 0};
        break;
      }
      if (f >= F.WB[r] && f < F.WB[r] + 8) {
        const int t = (f - F.WB[r]) >> 1, s = (f - F.WB[r]) & 1;
        o = FragSrc{We + (long long)(16 * t + m) * EDGE_IN + HID, 1, 0, s, 0};
        break;
      }
      if (f >= F.WC[r] && f < F.WC[r] + 4) {
        const int t = f - F.WC[r];
        o = FragSrc{We + (long long)(16 * t + m) * EDGE_IN + 2 * HID, 1, 2, 0, 0};
        break;
      }
      if (f >= F.WN[r] && f < F.WN[r] + 16) {  // k-steps 0, 1: h; 2, 3: aggregate
        const int t = (f - F.WN[r]) >> 2, s = (f - F.WN[r]) & 3;
        o = FragSrc{Wn + (long long)(16 * t + m) * NODE_IN + (s < 2 ? 0 : HID), 1, 0, s & 1, 0};
        break;
      }
      if (f >= F.WAT[r] && f < F.WAT[r] + 8) {
        const int t = (f - F.WAT[r]) >> 1, s = (f - F.WAT[r]) & 1;
        o = FragSrc{We + 16 * t + m, EDGE_IN, 0, s, 0};
        break;
      }
      if (f >= F.WBT[r] && f < F.WBT[r] + 8) {
        const int t = (f - F.WBT[r]) >> 1, s = (f - F.WBT[r]) & 1;
        o = FragSrc{We + HID + 16 * t + m, EDGE_IN, 0, s, 0};
        break;
      }
      if (f >= F.WNT[r] && f < F.WNT[r] + 16) {  // 8 row tiles (h then a) x 2 k-steps
        const int t = (f - F.WNT[r]) >> 1, s = (f - F.WNT[r]) & 1;
        o = FragSrc{Wn + 16 * t + m, NODE_IN, 0, s, 0};
        break;
      }
    }
  }
  return o;
}

// Blob position of value j of lane group q, or -1 for padding.
__host__ __device__ inline long long frag_index(const FragSrc &o, int q, int j) {
  switch (o.kind) {
    case 0:
      return o.base + (long long)o.stride * frag_channel(o.s, q, j);
    case 1: {
      const int k = 8 * q + j;
      return k < o.lim ? o.base + (long long)o.stride * k : -1LL;
    }
    case 2:
      return (q == 0 && j < 2) ? o.base + j : -1LL;
    default:
      return -1LL;
  }
}

__device__ __forceinline__ long long bias_index(const BlobLayout &L, const FragLayout &F, int R,
                                                int b, int lane, int e) {
  int q = lane >> 4;
  if (b == F.BH) {
    int k = 4 * q + e;
    return k < NOUT ? (long long)(L.bh + k) : -1LL;
  }
  int t, base;
  if (b >= F.B1 && b < F.B1 + 4) {
    t = b - F.B1;
    base = (int)L.b1;
  } else if (b >= F.B2 && b < F.B2 + 4) {
    t = b - F.B2;
    base = (int)L.b2;
  } else {
    base = -1;
    t = 0;
    for (int r = 0; r < R; ++r) {
      if (b >= F.BE[r] && b < F.BE[r] + 4) {
        t = b - F.BE[r];
        base = (int)L.be[r];
      }
      if (b >= F.BN[r] && b < F.BN[r] + 4) {
        t = b - F.BN[r];
        base = (int)L.bn[r];
      }
    }
    if (base < 0) return -1LL;
  }
  return (long long)(base + 16 * t + 4 * q + e);
}

__global__ __launch_bounds__(64) void gnn_prep_kernel(const float *__restrict__ blob, int R,
                                                      BlobLayout L, FragLayout F,
                                                      uint8_t *__restrict__ pack,
                                                      unsigned *__restrict__ ctrl) {
  int lane = threadIdx.x, f = blockIdx.x;
  // the fallback gate's arrival counts start every step at zero
  if (ctrl && f == 0 && lane == 0) {
    ctrl[1] = 0u;
    ctrl[2] = 0u;
  }
  // and so do the tile counters of the rounds and the chunk counters
  if (ctrl && f == 0 && lane < MAX_ROUNDS) ctrl[kCtrlTileQueue + lane] = 0u;
  if (ctrl && f == 0 && lane < kQueueParts) ctrl[kCtrlChunkQueue + kQueueStride * lane] = 0u;
  if (f < F.nfrag) {
    const FragSrc fs = frag_src(L, F, R, f, lane & 15);
    long long ix[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) ix[j] = frag_index(fs, lane >> 4, j);
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {  // padding loads blob[0] and discards it
      const float val = blob[ix[j] >= 0 ? ix[j] : 0];
      x[j] = ix[j] >= 0 ? val : 0.0f;
    }
    u32x4 v;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = pack_bf16(x[2 * k], x[2 * k + 1]);
    v = u32x4{w[0], w[1], w[2], w[3]};
    ((u32x4 *)(pack + F.frag_off))[(size_t)f * 64 + lane] = v;
  } else if (f < F.nfrag + F.nbias) {
    int b = f - F.nfrag;
    long long ix[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) ix[e] = bias_index(L, F, R, b, lane, e);
    float x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float val = blob[ix[e] >= 0 ? ix[e] : 0];
      x[e] = ix[e] >= 0 ? val : 0.0f;
    }
    f32x4 v;
    v.x = x[0];
    v.y = x[1];
    v.z = x[2];
    v.w = x[3];
    ((f32x4 *)(pack + F.bias_off))[(size_t)b * 64 + lane] = v;
  } else if (lane < 25) {
    ((float *)(pack + F.const_off))[lane] = blob[L.mu + lane];
  }
}

// ------------------------------------------------------------ encoder ---

// Shifted populations of node (x, y) of lattice `lat`: pulled through one
// streaming step from a post-collision state, or read in place.
template <bool PULL>
__device__ __forceinline__ void node_pops(const float *__restrict__ lat, int nx, int ny, int x,
                                          int y, float (&g)[9]) {
  if constexpr (PULL) {
    lbm::pull9(lat, nx, ny, x, y, g);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = lat[lbm::pidx(nx, y, i, x)];
  }
}

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// One wave per chunk of 64 consecutive nodes of a lattice row, chunks drawn
// from a grid-wide counter (ChunkQueue).  Per node (one lane each): the
// coalesced pull of the nine populations, the moments and the 12 normalised
// features, rounded to BF16 into the node's LDS slot (16 BF16, the last four
// zero).  The two layers then run on MFMA over four column blocks of 16 nodes,
// lane (n, q) = (node, channel group), reading the B operand from the slots:
// group q < 2 takes features 8q..8q+7.  Lanes past the row end (ragged nx)
// load a valid node and store nothing.
template <bool PULL, bool SAVE>
__global__ __launch_bounds__(kThreads, SAVE ? 3 : 4) void gnn_encode_kernel(
    const float *__restrict__ g, int batch, int nx, int ny, const uint8_t *__restrict__ pack,
    FragLayout F, uint16_t *__restrict__ h0, uint16_t *__restrict__ save_x,
    uint16_t *__restrict__ save_e1, unsigned *__restrict__ chunkq) {
  __shared__ __attribute__((aligned(16))) uint32_t slot_s[kWaves][64 * 8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
  const f32x4 *bias = (const f32x4 *)(pack + F.bias_off);
  const float *cst = (const float *)(pack + F.const_off);
  u32x4 w1[4], w2[4][2];
  f32x4 b1[4], b2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    w1[t] = load_frag(frags, F.W1 + t, lane);
    w2[t][0] = load_frag(frags, F.W2 + 2 * t, lane);
    w2[t][1] = load_frag(frags, F.W2 + 2 * t + 1, lane);
    b1[t] = load_bias(bias, F.B1 + t, lane);
    b2[t] = load_bias(bias, F.B2 + t, lane);
  }
  float mu[NFEAT], isg[NFEAT];
#pragma unroll
  for (int k = 0; k < NFEAT; ++k) {
    mu[k] = cst[C_MU + k];
    isg[k] = 1.0f / cst[C_SIGMA + k];
  }
  uint32_t *sw = slot_s[__builtin_amdgcn_readfirstlane(wave)];

  for (ChunkQueue cw(batch, nx, ny, kWaves, wave, chunkq); cw.more(); cw.next()) {
    const int xc = cw.xc, y = cw.y, b = cw.b;
    const float *lat = g + (size_t)b * ny * 9 * nx;
    {
      const int x = xc * 64 + lane;
      const unsigned drawn = cw.draw();
      float gp[9];
      node_pops<PULL>(lat, nx, ny, x < nx ? x : nx - 1, y, gp);
      float drho, rho, u, v, uu;
      lbm::node_moments(gp, drho, rho, u, v, uu);
      cw.take(drawn);
      const float raw[NFEAT] = {gp[0], gp[1], gp[2], gp[3], gp[4], gp[5],
                                gp[6], gp[7], gp[8], drho, u,     v};
      float ft[NFEAT];
#pragma unroll
      for (int k = 0; k < NFEAT; ++k) ft[k] = (raw[k] - mu[k]) * isg[k];
      u32x4 *o = (u32x4 *)(sw + lane * 8);
      o[0] = u32x4{pack_bf16(ft[0], ft[1]), pack_bf16(ft[2], ft[3]), pack_bf16(ft[4], ft[5]),
                   pack_bf16(ft[6], ft[7])};
      o[1] = u32x4{pack_bf16(ft[8], ft[9]), pack_bf16(ft[10], ft[11]), 0u, 0u};
    }
    wave_lds_sync();
#pragma unroll 1
    for (int grp = 0; grp < 4; ++grp) {
      const u32x4 xb = q < 2 ? *(const u32x4 *)(sw + (16 * grp + n) * 8 + 4 * q)
                             : u32x4{0u, 0u, 0u, 0u};
      f32x4 a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = gelu4(mfma(w1[t], xb, b1[t]));
      u32x4 e1[2] = {frag_from_acc(a[0], a[1]), frag_from_acc(a[2], a[3])};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 acc = mfma(w2[t][0], e1[0], b2[t]);
        a[t] = gelu4(mfma(w2[t][1], e1[1], acc));
      }
      u32x4 hb[2] = {frag_from_acc(a[0], a[1]), frag_from_acc(a[2], a[3])};
      const int x = xc * 64 + 16 * grp + n;
      if (x < nx) {
        size_t node = ((size_t)b * ny + y) * nx + x;
        u32x4 *dst = (u32x4 *)(h0 + node * HID);
        dst[q] = hb[0];
        dst[4 + q] = hb[1];
        if constexpr (SAVE) {
          if (q < 2) ((u32x4 *)(save_x + node * 16))[q] = xb;
          u32x4 *de = (u32x4 *)(save_e1 + node * HID);
          de[q] = e1[0];
          de[4 + q] = e1[1];
        }
      }
    }
    wave_lds_sync();
  }
}

// ------------------------------------------------- message passing round ---

constexpr int TILE_X = 16;              // receivers per tile row (one MFMA column block)
constexpr int TILE_Y = 8;               // tile rows
constexpr int HALO_X = TILE_X + 2;      // node states of the tile and its 1-node ring
constexpr int HALO_Y = TILE_Y + 2;
constexpr int HNODES = HALO_X * HALO_Y;

// LDS node stride: 128 B of state + 16 B of padding.  16 lanes reading the
// same 16-byte chunk of 16 consecutive nodes then touch 16 disjoint groups of
// 4 banks (144 B = 36 banks apart, mod 64), so the reads are conflict-free,
// and the address of a neighbour's chunk is the lane's own address plus a
// compile-time offset.
constexpr int kNodeBytes = 144;

__device__ __forceinline__ int wrapi(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

struct HeadArgs {
  const float *src;       // populations the collision starts from
  float *dst;             // corrected post-collision populations
  const float *tau_arr;   // per-lattice tau (device) or NULL
  float tau;              // tau when tau_arr is NULL
  float *head_out;        // [N][10] head outputs or NULL
  float *save_z;          // [N][12] head outputs kept for the backward pass
  double *pmass;          // [gridDim.x] FP64 sum of g* over the nodes of a workgroup
  unsigned *pflag;        // [gridDim.x] 1 if a population came out negative / non-finite
  GateArgs gate;          // the fallback gate (gate.ctrl NULL: none)
};

// Corrected collision of one node (Eq. 3 with the projected correction),
// populations I0 .. I1 - 1 (the moments and the projection use all nine).
template <int I0 = 0, int I1 = 9>
__device__ __forceinline__ void gnn_collide(float (&g)[9], const float (&z)[NOUT], float tau,
                                           float sdelta) {
  float drho, rho, u, v, uu;
  lbm::node_moments(g, drho, rho, u, v, uu);
  float sig = 1.0f / (1.0f + expf(-z[0]));
  float tau_adj = 0.5f + sig;
  float omega = 1.0f / (tau * tau_adj);
  float m0 = 0.0f, mx = 0.0f, my = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    m0 += z[1 + i];
    mx += float(cx(i)) * z[1 + i];
    my += float(cy(i)) * z[1 + i];
  }
  m0 *= (1.0f / 9.0f);
  mx *= (1.0f / 6.0f);
  my *= (1.0f / 6.0f);
#pragma unroll
  for (int i = I0; i < I1; ++i) {
    float relaxed = g[i] + omega * (lbm::geq_shifted<float>(i, drho, rho, u, v, uu) - g[i]);
    float df = z[1 + i] - m0 - float(cx(i)) * mx - float(cy(i)) * my;
    g[i] = relaxed + sdelta * df;
  }
}

// One round over 16 x 8 receiver tiles drawn from a counter, two 4-wave
// workgroups per CU.  The node states of a tile and its ring (18 x 10 nodes,
// BF16) sit in LDS; wave w handles tile rows 2w and 2w + 1, 16 receivers (one
// MFMA column block) at a time.  Two halo buffers alternate: while the waves
// work on one tile, direct-to-LDS loads (global_load_lds_dwordx4, no
// registers) fill the other with the next tile's halo, so fetching the node
// states overlaps the arithmetic instead of stalling it.  Two buffers and the
// weights take 76 KB, so two workgroups share a CU and each fills the other's
// barrier waits.  With HEAD the round is the last one: the head, the
// projection and the corrected collision follow, written to args.dst; the
// head outputs pass through the buffer the tile has just been computed from.
// Register budget (two waves per SIMD): only the sender weights Wb, used 8
// times per receiver, stay in VGPRs; Wa, Wn, the head and the biases are read
// from LDS where they are used.
constexpr int kRoundThreads = 256;
constexpr int kRoundWaves = kRoundThreads / 64;
constexpr int kRowsPerWave = TILE_Y / kRoundWaves;
// A halo buffer is a run of 16-byte slots, node ln's chunk c at slot 9 ln + c
// (slot 9 ln + 8 is the padding of kNodeBytes); one direct-to-LDS load fills
// 64 consecutive slots.
constexpr int kStageLoads = (HNODES * 9 + 63) / 64;
constexpr int kStagePerWave = (kStageLoads + kRoundWaves - 1) / kRoundWaves;
constexpr int kHaloBytes = kStageLoads * 64 * 16;
static_assert(kNodeBytes == 9 * 16, "a node is nine 16-byte slots");
static_assert(kRowsPerWave * kRoundWaves == TILE_Y, "tile rows split over the waves");
static_assert(TILE_X * TILE_Y * NOUT * 4 <= kHaloBytes, "head outputs fit in a halo buffer");
static_assert((16 + 4) * kRoundThreads <= kHaloBytes, "reduction fits in a halo buffer");
// Divisions of the staging loop by multiply and shift (full-rate 24-bit
// multiplies): slot / 9 for every slot of a halo buffer and node / HALO_X for
// every node, checked here over the whole range.
constexpr int kDiv9Mul = 7282, kDivHaloMul = 3641;
constexpr bool magic_divisions_exact() {
  for (int v = 0; v < kStageLoads * 64; ++v)
    if (((v * kDiv9Mul) >> 16) != v / 9) return false;
  for (int v = 0; v < HNODES; ++v)
    if (((v * kDivHaloMul) >> 16) != v / HALO_X) return false;
  return true;
}
static_assert(HALO_X == 18 && magic_divisions_exact(), "staging divisions");

// s_waitcnt with vmcnt(0) and the other counters left at their maximum: waits
// for this wave's vector memory operations only (the stores counted too).
constexpr int kWaitVmcnt0 = 0x0F70;

// Workgroup barrier that makes this wave's LDS writes visible (lgkmcnt(0))
// but does not wait for its global stores.  __syncthreads() cannot be used
// inside the tile loop: with direct-to-LDS loads in the kernel its release
// fence waits for every vector memory operation, the fresh stores of the
// tile included.  The loads into LDS are waited for explicitly
// (kWaitVmcnt0) before the barrier that publishes them; the memory clobber
// keeps the compiler from moving memory accesses across the barrier.
// Stores a row's fragments (chunks q and 4 + q of the node in lane 16 q + n)
// through a raw buffer resource of `bytes` bytes at `base`: stores at
// offsets past the range are dropped by the hardware.
constexpr int kNodeStateBytes = HID * 2;
constexpr int kBufferRsrcWord3 = 0x00020000;
typedef int i32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_row(uint16_t *base, int bytes, int off, const u32x4 (&v)[2]) {
  // base and bytes are wave-uniform; saying so keeps the resource in scalar
  // registers (no per-lane loop over resources)
  const uint64_t pb = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)pb);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(pb >> 32));
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(((uint64_t)hi << 32) | lo), 0, __builtin_amdgcn_readfirstlane(bytes),
      kBufferRsrcWord3);
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4_t, v[0]), rs, off, 0, 0);
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4_t, v[1]), rs, off + 64, 0, 0);
}

__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <bool HEAD, bool PULL, bool SAVE>
__global__ __launch_bounds__(kRoundThreads, 2) void gnn_round_kernel(
    const uint16_t *__restrict__ hin, uint16_t *__restrict__ hout,
    uint16_t *__restrict__ save_agg, int batch, int nx, int ny, int round,
    const uint8_t *__restrict__ pack, FragLayout F, HeadArgs args, unsigned *__restrict__ tileq) {
  __shared__ __attribute__((aligned(16))) uint8_t hs_a[kHaloBytes];
  __shared__ __attribute__((aligned(16))) uint8_t hs_b[kHaloBytes];
  __shared__ u32x4 wa_s[8 * 64];
  __shared__ u32x4 wn_s[16 * 64];

  // the wave index is wave-uniform; saying so keeps what derives from it (tile
  // rows, the staging loop) in scalar registers
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int n = lane & 15, q = lane >> 4;
  const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
  const f32x4 *bias = (const f32x4 *)(pack + F.bias_off);
  const float *cst = (const float *)(pack + F.const_off);

  for (int k = threadIdx.x; k < 8 * 64; k += kRoundThreads)
    wa_s[k] = frags[(size_t)F.WA[round] * 64 + k];
  for (int k = threadIdx.x; k < 16 * 64; k += kRoundThreads)
    wn_s[k] = frags[(size_t)F.WN[round] * 64 + k];
  u32x4 wb[4][2];
  uint32_t wc[4];  // only lanes q == 0 hold a non-zero (first) dword
  f32x4 be[4], bn[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    wb[t][0] = load_frag(frags, F.WB[round] + 2 * t, lane);
    wb[t][1] = load_frag(frags, F.WB[round] + 2 * t + 1, lane);
    wc[t] = load_frag(frags, F.WC[round] + t, lane).x;
    be[t] = load_bias(bias, F.BE[round] + t, lane);
    bn[t] = load_bias(bias, F.BN[round] + t, lane);
  }
  float sdelta = 0.0f;
  u32x4 wh[2];
  f32x4 bh;
  if constexpr (HEAD) {
    wh[0] = load_frag(frags, F.WH, lane);
    wh[1] = load_frag(frags, F.WH + 1, lane);
    bh = load_bias(bias, F.BH, lane);
    sdelta = cst[C_SDELTA];
  }

  const int txn = (nx + TILE_X - 1) / TILE_X, tyn = (ny + TILE_Y - 1) / TILE_Y;
  const long long ntiles = (long long)batch * txn * tyn;

  struct TileAt {
    int x0, y0, b;
    size_t lat_nodes;
  };
  auto tile_at = [&](long long tile) {
    TileAt T;
    const int tx = (int)(tile % txn);
    const long long rest = tile / txn;
    const int ty = (int)(rest % tyn);
    T.b = (int)(rest / tyn);
    T.x0 = tx * TILE_X;
    T.y0 = ty * TILE_Y;
    T.lat_nodes = (size_t)T.b * ny * nx;
    return T;
  };

  // Byte offset from the halo's first node of the 16 bytes that slot
  // `slot` of a halo buffer takes in an interior tile: chunk c of halo node
  // ln = (hx, hy), at (hy nx + hx) 128 + 16 c, with 24-bit multiplies
  // (nx <= 2^20 keeps it in 32 bits; larger lattices take the general path).
  const bool stage_interior_ok = nx <= (1 << 20);
  auto stage_offset = [&](unsigned slot) -> unsigned {
    unsigned ln = __umul24(slot, kDiv9Mul) >> 16;
    unsigned c = slot - 9 * ln;
    if (ln >= (unsigned)HNODES) {
      ln = HNODES - 1;
      c = 7;
    }
    c = c < 7 ? c : 7;
    const unsigned hy = __umul24(ln, kDivHaloMul) >> 16;
    const unsigned hx = ln - HALO_X * hy;
    return (__umul24(hy, (unsigned)nx) + hx) * 128u + c * 16u;
  };
  // Without the head the kernel has the registers to compute this lane's
  // offsets once (load k = wave + 4 i fills slot 64 k + lane, the same in
  // every interior tile), which takes the address arithmetic out of the tile
  // loop (-2 % of the round); the last round computes them per tile.
  unsigned stage_off[kStagePerWave];
#pragma unroll
  for (int i = 0; i < kStagePerWave; ++i) {
    const int k = wave + kRoundWaves * i;
    stage_off[i] = HEAD ? 0u : stage_offset(64u * (k < kStageLoads ? k : 0) + lane);
  }

  // Issues the direct-to-LDS loads of a tile's halo into `buf`: load k of
  // this wave fills slots 64 k .. 64 k + 63, lane l slot 64 k + l.  Padding
  // slots take a copy of chunk 7, slots past the last node a copy of the last
  // node: every address is a valid node state, every slot inside `buf`.
  auto stage = [&](long long tile, uint8_t *buf) {
    const TileAt T = tile_at(tile);
    // With the head, the lane index is recounted here (mbcnt) rather than
    // kept: held across the tile it was spilled to scratch, and reloading it
    // made every tile wait for all of the previous tile's stores.
    int sl = lane;
    if constexpr (HEAD) {
      asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(sl));
    }
    // Interior tiles (the halo wraps nowhere): the loads take the offsets
    // computed above from the halo's first node.
    if (T.x0 >= 1 && T.x0 + HALO_X - 1 <= nx && T.y0 >= 1 && T.y0 + HALO_Y - 1 <= ny &&
        stage_interior_ok) {
      const uint8_t *base =
          (const uint8_t *)(hin + (T.lat_nodes + (size_t)(T.y0 - 1) * nx + (T.x0 - 1)) * HID);
      if constexpr (HEAD) {
        for (int k = wave; k < kStageLoads; k += kRoundWaves)
          __builtin_amdgcn_global_load_lds(
              (const void *)(base + stage_offset(64u * k + sl)),
              (__attribute__((address_space(3))) void *)(buf + k * 1024), 16, 0, 0);
      } else {
#pragma unroll
        for (int i = 0; i < kStagePerWave; ++i) {
          const int k = wave + kRoundWaves * i;
          if (k < kStageLoads)
            __builtin_amdgcn_global_load_lds(
                (const void *)(base + stage_off[i]),
                (__attribute__((address_space(3))) void *)(buf + k * 1024), 16, 0, 0);
        }
      }
      return;
    }
    for (int k = wave; k < kStageLoads; k += kRoundWaves) {
      const int slot = 64 * k + sl;
      int ln = slot / 9;
      int c = slot - 9 * ln;
      if (ln >= HNODES) ln = HNODES - 1;
      if (c == 8) c = 7;
      const int hy = ln / HALO_X, hx = ln - hy * HALO_X;
      int gx = T.x0 - 1 + hx, gy = T.y0 - 1 + hy;
      gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
      gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
      if (gx >= nx) gx = wrapi(gx, nx);  // lattices narrower than the halo
      if (gy >= ny) gy = wrapi(gy, ny);
      const uint16_t *src = hin + (T.lat_nodes + (size_t)gy * nx + gx) * HID + c * 8;
      __builtin_amdgcn_global_load_lds(
          (const void *)src, (__attribute__((address_space(3))) void *)(buf + k * 1024), 16, 0,
          0);
    }
  };

  Q80 mass_acc{0ull, 0ll};
  unsigned flag_acc = 0;

  // The last row's stores of the previous tile (without the head), issued
  // once the barrier that starts a tile has passed.
  bool pend = false;
  size_t pend_row = 0;
  int pend_bytes = 0, pend_off = 0;
  u32x4 pend_hb[2] = {}, pend_ab[2] = {};
  auto release = [&]() {
    if constexpr (!HEAD) {
      if (pend) {
        if (hout) store_row(hout + pend_row * HID, pend_bytes, pend_off, pend_hb);
        if constexpr (SAVE) store_row(save_agg + pend_row * HID, pend_bytes, pend_off, pend_ab);
        pend = false;
      }
    }
  };

  // The receivers of one tile from the halo in `hs`; with HEAD the head
  // outputs then pass through `hs` itself (float zb[TILE_X * TILE_Y][NOUT]).
  auto compute = [&](const TileAt &T, uint8_t *hs) {
    const int x0 = T.x0, y0 = T.y0, b = T.b;
    const size_t lat_nodes = T.lat_nodes;
    // head outputs of the wave's two rows: row 0's in zr0, row 1's in zr1
    // (shifted along row by row; an array indexed by the row counter costs
    // a select per element and position)
    static_assert(kRowsPerWave == 2, "head outputs of two rows per wave");
    f32x4 zr0 = {}, zr1 = {};
#pragma unroll 1
    for (int r = 0; r < kRowsPerWave; ++r) {
      // An offset the compiler cannot see through, so that the LDS weight
      // reads below stay inside the loop instead of being hoisted into
      // registers (which would halve the waves per SIMD).
      int wo = lane;
      asm volatile("" : "+v"(wo));
      const u32x4 *wa = wa_s + wo, *wn = wn_s + wo;
      const int tyl = wave * kRowsPerWave + r;
      const int x = x0 + n, y = y0 + tyl;
      // chunk q of the lower-left neighbour (dx = dy = -1) of this receiver;
      // every neighbour's chunk is at a constant offset from it
      const uint8_t *nb = hs + (tyl * HALO_X + n) * kNodeBytes + q * 16;
      auto frag_at = [&](int dx, int dy, int s) {
        return *(const u32x4 *)(nb + ((dy + 1) * HALO_X + dx + 1) * kNodeBytes + s * 64);
      };
      // Every LDS read of the row's receiver part is issued before the first
      // wait: the receiver's state, the eight Wa fragments and the sender
      // states of the first two edges.
      u32x4 hn[2] = {frag_at(0, 0, 0), frag_at(0, 0, 1)};
      u32x4 waf[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) waf[k] = wa[k * 64];
      // sender states of edge e in hj[e & 1], read one edge ahead of use
      u32x4 hj[2][2];
      hj[1][0] = frag_at(cx(1), cy(1), 0);
      hj[1][1] = frag_at(cx(1), cy(1), 1);
      hj[0][0] = frag_at(cx(2), cy(2), 0);
      hj[0][1] = frag_at(cx(2), cy(2), 1);
      f32x4 an[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        an[t] = mfma(waf[2 * t], hn[0], be[t]);
        an[t] = mfma(waf[2 * t + 1], hn[1], an[t]);
      }
      f32x4 agg[4] = {};
      const uint32_t q0 = q == 0 ? 0xffffffffu : 0u;
      // Pre-activation of the message from direction d (MFMA only).
      auto message = [&](int d, const u32x4(&h)[2], f32x4(&acc)[4]) {
        const u32x4 ed = {q0 & (bf16_unit(cx(d)) | (bf16_unit(cy(d)) << 16)), 0u, 0u, 0u};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[t] = mfma(u32x4{wc[t], 0u, 0u, 0u}, ed, an[t]);
          acc[t] = mfma(wb[t][0], h[0], acc[t]);
          acc[t] = mfma(wb[t][1], h[1], acc[t]);
        }
      };
      // Software pipeline over the 8 edges: step d issues the LDS reads of
      // edge d + 2, the MFMA chains of edge d + 1 and the GELUs of edge d,
      // whose pre-activations were formed one step earlier.  A scheduling
      // barrier closes each step, so the compiler cannot move a chain next to
      // the GELUs that consume it (which would expose the MFMA latency);
      // inside a step each of the 12 MFMAs is followed by 8 VALU
      // instructions.  Summation order is unchanged.
      f32x4 acc[2][4];
      message(1, hj[1], acc[0]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int d = 1; d < 9; ++d) {
        if (d + 2 <= 8) {
          hj[d & 1][0] = frag_at(cx(d + 2), cy(d + 2), 0);
          hj[d & 1][1] = frag_at(cx(d + 2), cy(d + 2), 1);
        }
        if (d < 8) message(d + 1, hj[(d + 1) & 1], acc[d & 1]);
#pragma unroll
        for (int t = 0; t < 4; ++t) agg[t] += gelu4(acc[(d - 1) & 1][t]);
        if (d + 2 <= 8) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        if (d < 8) {
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      u32x4 ab[2] = {frag_from_acc(agg[0], agg[1]), frag_from_acc(agg[2], agg[3])};
      // Node update: the Wn fragments of row tile t + 1 are read while the
      // chain of row tile t runs.
      f32x4 p[4];
      u32x4 wnf[2][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) wnf[0][k] = wn[k * 64];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < 3) {
#pragma unroll
          for (int k = 0; k < 4; ++k) wnf[(t + 1) & 1][k] = wn[(4 * (t + 1) + k) * 64];
        }
        const u32x4(&w)[4] = wnf[t & 1];
        p[t] = mfma(w[0], hn[0], bn[t]);
        p[t] = mfma(w[1], hn[1], p[t]);
        p[t] = mfma(w[2], ab[0], p[t]);
        p[t] = mfma(w[3], ab[1], p[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) p[t] = gelu4(p[t]);
      u32x4 hb[2] = {frag_from_acc(p[0], p[1]), frag_from_acc(p[2], p[3])};
      // The row's stores go through buffer resources whose range ends at
      // the lattice edge (none for a row past it): the hardware drops the
      // lanes outside the lattice.  Without the head, the last row's stores
      // are held back until the barrier that starts the next tile has passed
      // (see the wait below).
      {
        const int yu = __builtin_amdgcn_readfirstlane(y);
        const bool row_in = yu < ny;
        const size_t row0 = lat_nodes + (size_t)(row_in ? yu : ny - 1) * nx + x0;
        const int bytes = row_in ? (nx - x0) * kNodeStateBytes : 0;
        const int off = n * kNodeStateBytes + q * 16;
        if (HEAD || r + 1 < kRowsPerWave) {
          if (hout) store_row(hout + row0 * HID, bytes, off, hb);
          if constexpr (SAVE) store_row(save_agg + row0 * HID, bytes, off, ab);
        } else {
          pend = true;
          pend_row = row0;
          pend_bytes = bytes;
          pend_off = off;
          pend_hb[0] = hb[0];
          pend_hb[1] = hb[1];
          pend_ab[0] = ab[0];
          pend_ab[1] = ab[1];
        }
      }
      if constexpr (HEAD) {
        f32x4 z = mfma(wh[0], hb[0], bh);
        zr0 = zr1;
        zr1 = mfma(wh[1], hb[1], z);
      }
    }

    // This wave's direct-to-LDS loads of the next tile's halo, issued before
    // its rows, must be complete before the barrier that starts the next
    // tile.  At this point only they, the stores released at the start of
    // the tile and the first row's stores are in flight, all issued at least
    // a row earlier, so the wait seldom stalls; the last row's stores, held
    // back, drain while the next tile is computed.  A wait in every row,
    // before its stores, cost a tenth of the round.
    if constexpr (!HEAD) __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);

    if constexpr (HEAD) {
      // the halo loads are complete before the epilogue's own loads and
      // stores are issued
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      // The collision of the tile's 128 nodes: waves 2j and 2j + 1 take nodes
      // 64 j .. 64 j + 63, one per lane, and split the nine populations
      // between them (0-4 and 5-8), so every lane of every wave works.  The
      // populations are loaded first, so that their latency passes while the
      // head outputs are exchanged (lanes past the lattice edge load a valid
      // node and store nothing).
      const int nl = (wave >> 1) * 64 + lane;
      const int tyl = nl / TILE_X, nxl = nl - tyl * TILE_X;
      const int x = x0 + nxl, y = y0 + tyl;
      const bool inside = x < nx && y < ny;
      const size_t lat_off = (size_t)b * ny * 9 * nx;
      float gp[9];
      node_pops<PULL>(args.src + lat_off, nx, ny, inside ? x : x0, inside ? y : y0, gp);
      // every wave is done reading the halo: its buffer takes the head outputs
      float *zb = (float *)hs;
      lds_barrier();
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) {
        const int tyl = wave * kRowsPerWave + r;
        const f32x4 zv = r == 0 ? zr0 : zr1;
        const float zz[4] = {zv.x, zv.y, zv.z, zv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int k = 4 * q + e;
          if (k < NOUT) zb[(tyl * TILE_X + n) * NOUT + k] = zz[e];
        }
      }
      lds_barrier();
      const bool lo = (wave & 1) == 0;
      static_assert(TILE_X * TILE_Y == 2 * 64 && kRoundWaves == 4, "epilogue split");
      double msum = 0.0;
      unsigned bad = 0;
      // Every lane collides (lanes past the edge hold a valid node), so the
      // loaded populations are consumed on every path; only the stores depend
      // on `inside`.  With the collision inside the branch, the compiler saw a
      // path on which the loads were still in flight at the next tile and
      // waited for all memory operations at the first row of every other
      // tile, the next tile's halo loads included.
      float z[NOUT];
#pragma unroll
      for (int k = 0; k < NOUT; ++k) z[k] = zb[nl * NOUT + k];
      const float tau = args.tau_arr ? args.tau_arr[b] : args.tau;
      if (lo)
        gnn_collide<0, 5>(gp, z, tau, sdelta);
      else
        gnn_collide<5, 9>(gp, z, tau, sdelta);
      if (inside) {
        float *d = args.dst + lat_off + (size_t)y * 9 * nx + x;
        auto finish = [&](int i) {
          __builtin_nontemporal_store(gp[i], d + (size_t)i * nx);
          float f = gp[i] + lbm::wgt<float>(i);
          bad |= (f >= 0.0f && f < INFINITY) ? 0u : 1u;
          msum += (double)gp[i];
        };
        if (lo) {
#pragma unroll
          for (int i = 0; i < 5; ++i) finish(i);
        } else {
#pragma unroll
          for (int i = 5; i < 9; ++i) finish(i);
        }
        const size_t node = lat_nodes + (size_t)y * nx + x;
        if (lo && args.head_out)
          for (int k = 0; k < NOUT; ++k) args.head_out[node * NOUT + k] = z[k];
        if constexpr (SAVE)
          if (lo)
            for (int k = 0; k < NOUT; ++k) args.save_z[node * 12 + k] = z[k];
      }
      // Exact fixed-point accumulation: the gate's total does not depend on
      // which workgroup drew which tile.
      mass_acc = q80_add(mass_acc, q80_of(msum));
      flag_acc |= bad;
    }
  };

  // Tile i of this workgroup works from hs_a when i is even and from hs_b
  // when odd; each half of the loop names its buffers directly, so the
  // compiler can tell the LDS reads of one buffer from the loads in flight
  // into the other.  Every wave has waited for its own loads into the current
  // buffer (below for the first tile, inside the previous tile's work for the
  // others); the barrier at the top of each half makes all of them visible
  // and tells that the other buffer is no longer read.
  //
  // Tile order: the first two tiles of a workgroup are blockIdx.x and
  // blockIdx.x + gridDim.x; every later one comes from a counter shared by
  // the grid (zeroed by the weight packing each step), so that the two
  // workgroups sharing a CU finish together even though the older one's
  // waves are issued first (with a fixed assignment the younger one ran on
  // alone for the last 40 % of the round).  Thread 0 draws the tile after
  // next while the current one is computed and passes it on through `qslot`.
  // Which workgroup computes a tile changes nothing in its results.
  constexpr bool kQueue = true;
  __shared__ long long qslot[2];
  const long long g = gridDim.x;
  unsigned drawn = 0;
  auto draw = [&](long long nxt) {
    if (kQueue && threadIdx.x == 0 && nxt < ntiles) {
      // An address the compiler cannot prove wave-uniform: otherwise it
      // rewrites the one-lane atomic into a wave-wide one and waits for its
      // result at once, instead of where the result is used.
      int z = 0;
      asm volatile("" : "+v"(z));
      drawn = atomicAdd(tileq + z, 1u);
    }
  };
  auto after_next = [&](long long nxt) -> long long {
    if (nxt >= ntiles) return ntiles;
    return kQueue ? 2 * g + (long long)drawn : nxt + g;
  };
  long long tile = blockIdx.x;
  if (threadIdx.x == 0) qslot[1] = tile + g;
  if (tile < ntiles) stage(tile, hs_a);
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  while (tile < ntiles) {
    lds_barrier();
    long long next = qslot[1];
    release();
    if (next < ntiles) stage(next, hs_b);
    draw(next);
    compute(tile_at(tile), hs_a);
    if (threadIdx.x == 0) qslot[0] = after_next(next);
    tile = next;
    if (tile >= ntiles) break;
    lds_barrier();
    next = qslot[0];
    release();
    if (next < ntiles) stage(next, hs_a);
    draw(next);
    compute(tile_at(tile), hs_b);
    if (threadIdx.x == 0) qslot[1] = after_next(next);
    tile = next;
  }
  release();

  if constexpr (HEAD) {
    __syncthreads();  // last tile's head outputs consumed
    Q80 *red_m = (Q80 *)hs_a;
    unsigned *red_f = (unsigned *)(hs_a + sizeof(Q80) * kRoundThreads);
    red_m[threadIdx.x] = mass_acc;
    red_f[threadIdx.x] = flag_acc;
    __syncthreads();
    for (int s = kRoundThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        red_m[threadIdx.x] = q80_add(red_m[threadIdx.x], red_m[threadIdx.x + s]);
        red_f[threadIdx.x] |= red_f[threadIdx.x + s];
      }
      __syncthreads();
    }
    Q80 *pmass = (Q80 *)args.pmass;
    if (threadIdx.x == 0) {
      pmass[blockIdx.x] = red_m[0];
      args.pflag[blockIdx.x] = red_f[0];
    }
    if constexpr (PULL) {
      if (args.gate.ctrl)
        gate_decide_last<kRoundThreads>(args.gate, pmass, args.pflag, (int)gridDim.x,
                                        (double)batch * nx * ny, red_m, red_f);
    }
  }
}

// ------------------------------------------------------------ fallback ---

// Plain BGK step from the unchanged source when the gate tripped (same
// arithmetic as bgk_pull_kernel, grid-stride; for the channel, the same as
// channel_pull_kernel: walls and forcing); exits at once otherwise.  The
// workgroup that finishes last sums the FP64 partials of what was stored in
// index order and records it as the new total mass.
__global__ __launch_bounds__(kThreads) void gate_fallback_kernel(
    const float *__restrict__ src, float *__restrict__ dst, int nx, int ny, float omega,
    int walls, float gx, unsigned *__restrict__ ctrl, double *__restrict__ pmass2,
    double *__restrict__ mass) {
  __shared__ double sm[kThreads];
  __shared__ unsigned last_s;
  if (ctrl[0] == 0) return;
  double m = 0.0;
  const size_t nodes = (size_t)nx * ny;
  for (size_t k = (size_t)blockIdx.x * kThreads + threadIdx.x; k < nodes;
       k += (size_t)gridDim.x * kThreads) {
    int x = (int)(k % nx), y = (int)(k / nx);
    float g[9];
    if (walls) {
      lbm::pull9_walls(src, nx, ny, x, y, g);
      lbm::forced_collide(g, omega, gx);
    } else {
      lbm::pull9(src, nx, ny, x, y, g);
      lbm::bgk_collide(g, omega);
    }
    float *d = dst + (size_t)y * 9 * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      d[(size_t)i * nx] = g[i];
      m += (double)g[i];
    }
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pmass2[blockIdx.x] = sm[0];
    __threadfence();  // the partial before the arrival
    const unsigned done = atomicAdd(&ctrl[2], 1u);
    last_s = done == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (!last_s) return;
  __threadfence();  // every other workgroup's partial is visible
  m = 0.0;
  for (int k = threadIdx.x; k < (int)gridDim.x; k += kThreads) m += pmass2[k];
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *mass = (double)nodes + sm[0];
}

}  // namespace gnn

// ------------------------------------------------------------------- ABI ---

using namespace gnn;
using lbm::check_device;
using lbm::fail;
using lbm::launch_check;

// Workgroups of the encoder resident per CU (every instance has the same
// register budget; the occupancy query needs a current device).
static int encode_blocks_per_cu() {
  static int cached = 0;
  if (cached == 0) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &v, reinterpret_cast<const void *>(&gnn_encode_kernel<true, false>), kThreads, 0) !=
            hipSuccess ||
        v <= 0)
      v = 2;
    cached = v;
  }
  return cached;
}

static int device_cus() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v <= 0)
      v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

static inline void *at(void *base, size_t off) { return (uint8_t *)base + off; }

extern "C" size_t gnn_param_count(int n_rounds) {
  if (n_rounds < 0 || n_rounds > MAX_ROUNDS) return 0;
  return blob_layout(n_rounds).nparam;
}
extern "C" size_t gnn_blob_len(int n_rounds) {
  if (n_rounds < 0 || n_rounds > MAX_ROUNDS) return 0;
  return blob_layout(n_rounds).total;
}

namespace gnn {

int launch_prep(const float *params, int R, uint8_t *pack, unsigned *ctrl, hipStream_t s) {
  const BlobLayout L = blob_layout(R);
  const FragLayout F = frag_layout(R);
  if (F.total > kPackBytes) return fail(LBM_EINVAL, "packed weights exceed their scratch");
  hipLaunchKernelGGL(gnn_prep_kernel, dim3(F.nfrag + F.nbias + 1), dim3(64), 0, s, params, R, L,
                     F, pack, ctrl);
  return launch_check("gnn_prep_kernel");
}

// Launches weight packing, encoder and rounds.  src: populations the
// collision starts from (post-collision state of the previous step when
// PULL, else pre-collision); the last round writes dst and the partials.
int launch_forward(bool pull, const float *src, float *dst, int batch, int nx, int ny,
                   const float *tau_arr, float tau, const float *params, int R, float *head_out,
                   void *saved, void *ws, const lbm_fallback *fb, hipStream_t s) {
  const long long nodes = (long long)batch * nx * ny;
  const FragLayout F = frag_layout(R);
  const ForwardScratch W = forward_scratch(nodes);
  uint8_t *pack = (uint8_t *)at(ws, W.pack);
  unsigned *ctrl = (unsigned *)at(ws, W.ctrl);
  if (int rc = launch_prep(params, R, pack, ctrl, s)) return rc;

  const int cus = device_cus();
  const bool save = saved != nullptr;
  SavedLayout S{};
  if (save) S = saved_layout(nodes, R);
  auto hbuf = [&](int r) -> uint16_t * {  // node states h_r
    if (save) return (uint16_t *)at(saved, S.h + (size_t)r * align256((size_t)nodes * HID * 2));
    return (uint16_t *)at(ws, (r & 1) ? W.hB : W.hA);
  };

  // the encoder's grid: the workgroups that fit on the device at once (four
  // per CU for inference, three when saving activations); their waves draw
  // the chunks from a counter, so a larger grid would only add workgroups
  // that start late
  long long chunks = (long long)batch * ny * ((nx + 63) / 64);
  long long eblocks = (chunks + kWaves - 1) / kWaves;
  const long long eres = (long long)cus * encode_blocks_per_cu();
  int eb = (int)(eblocks < eres ? eblocks : eres);
  uint16_t *sx = save ? (uint16_t *)at(saved, S.x) : nullptr;
  uint16_t *se = save ? (uint16_t *)at(saved, S.e1) : nullptr;
  if (pull) {
    hipLaunchKernelGGL((gnn_encode_kernel<true, false>), dim3(eb), dim3(kThreads), 0, s, src,
                       batch, nx, ny, pack, F, hbuf(0), sx, se, ctrl + kCtrlChunkQueue);
  } else if (save) {
    hipLaunchKernelGGL((gnn_encode_kernel<false, true>), dim3(eb), dim3(kThreads), 0, s, src,
                       batch, nx, ny, pack, F, hbuf(0), sx, se, ctrl + kCtrlChunkQueue);
  } else {
    hipLaunchKernelGGL((gnn_encode_kernel<false, false>), dim3(eb), dim3(kThreads), 0, s, src,
                       batch, nx, ny, pack, F, hbuf(0), sx, se, ctrl + kCtrlChunkQueue);
  }
  if (int rc = launch_check("gnn_encode_kernel")) return rc;

  long long ntiles =
      (long long)batch * ((nx + TILE_X - 1) / TILE_X) * ((ny + TILE_Y - 1) / TILE_Y);
  long long cap = (long long)cus * 2;
  if (cap > kMaxGnnBlocks) cap = kMaxGnnBlocks;
  int rb = (int)(ntiles < cap ? ntiles : cap);
  HeadArgs none{};
  HeadArgs ha{};
  ha.src = src;
  ha.dst = dst;
  ha.tau_arr = tau_arr;
  ha.tau = tau;
  ha.head_out = head_out;
  ha.save_z = save ? (float *)at(saved, S.z) : nullptr;
  ha.pmass = (double *)at(ws, W.pmass);
  ha.pflag = (unsigned *)at(ws, W.pflag);
  if (fb && pull) ha.gate = GateArgs{ctrl, fb->drift_threshold, fb->flags, fb->n_fallback, fb->mass};
  for (int r = 0; r < R; ++r) {
    const bool head = r == R - 1;
    uint16_t *hin = hbuf(r);
    uint16_t *hout = head ? (save ? hbuf(r + 1) : nullptr) : hbuf(r + 1);
    uint16_t *sag = save ? (uint16_t *)at(saved, S.agg + (size_t)r * align256((size_t)nodes * HID * 2))
                         : nullptr;
    if (!head) {
      if (save)
        hipLaunchKernelGGL((gnn_round_kernel<false, false, true>), dim3(rb), dim3(kRoundThreads), 0,
                           s, hin, hout, sag, batch, nx, ny, r, pack, F, none, ctrl + kCtrlTileQueue + r);
      else
        hipLaunchKernelGGL((gnn_round_kernel<false, false, false>), dim3(rb), dim3(kRoundThreads), 0,
                           s, hin, hout, sag, batch, nx, ny, r, pack, F, none, ctrl + kCtrlTileQueue + r);
    } else if (pull) {
      hipLaunchKernelGGL((gnn_round_kernel<true, true, false>), dim3(rb), dim3(kRoundThreads), 0, s,
                         hin, hout, sag, batch, nx, ny, r, pack, F, ha, ctrl + kCtrlTileQueue + r);
    } else if (save) {
      hipLaunchKernelGGL((gnn_round_kernel<true, false, true>), dim3(rb), dim3(kRoundThreads), 0, s,
                         hin, hout, sag, batch, nx, ny, r, pack, F, ha, ctrl + kCtrlTileQueue + r);
    } else {
      hipLaunchKernelGGL((gnn_round_kernel<true, false, false>), dim3(rb), dim3(kRoundThreads), 0, s,
                         hin, hout, sag, batch, nx, ny, r, pack, F, ha, ctrl + kCtrlTileQueue + r);
    }
    if (int rc = launch_check("gnn_round_kernel")) return rc;
  }
  return LBM_OK;
}

}  // namespace gnn

namespace gnn {

// The fallback kernel of the per-step gate, after a corrected step whose last
// workgroup took the decision into ctrl[0]: recompute with plain BGK if
// tripped (the kernel exits at once otherwise) and record the new mass.
int launch_gate(const float *g_src, float *g_dst, int nx, int ny, float tau, int walls,
                float gx, const lbm_fallback *fb, void *pmass2, void *ctrl, hipStream_t s) {
  long long fbn = ((long long)nx * ny + kThreads - 1) / kThreads;
  int fbb = (int)(fbn < kMaxGnnBlocks ? fbn : kMaxGnnBlocks);
  hipLaunchKernelGGL(gate_fallback_kernel, dim3(fbb), dim3(kThreads), 0, s, g_src, g_dst, nx, ny,
                     1.0f / tau, walls, gx, (unsigned *)ctrl, (double *)pmass2, fb->mass);
  return launch_check("gate_fallback_kernel");
}

}  // namespace gnn

static int check_gnn_common(const char *who, int batch, int nx, int ny, const float *params,
                            int R) {
  if (!params) return fail(LBM_EINVAL, "%s: null parameters", who);
  if (R < 1 || R > MAX_ROUNDS) return fail(LBM_EINVAL, "%s: n_rounds %d not in [1, %d]", who, R,
                                           MAX_ROUNDS);
  if (batch < 1 || !lbm::lattice_ok(nx, ny) || (long long)batch * nx * ny >= (1LL << 31))
    return fail(LBM_EINVAL, "%s: bad sizes batch %d, %d x %d", who, batch, nx, ny);
  return LBM_OK;
}

extern "C" int gnn_forward(const float *g_pre, float *g_post, int batch, int nx, int ny,
                           const float *tau, const float *params, int n_rounds, float *head_out,
                           void *saved, size_t saved_bytes, void *workspace, size_t ws_bytes,
                           void *stream) {
  if (int rc = check_gnn_common("gnn_forward", batch, nx, ny, params, n_rounds)) return rc;
  if (!g_pre || !g_post || !tau) return fail(LBM_EINVAL, "gnn_forward: null pointer");
  size_t bytes = (size_t)batch * 9 * nx * ny * sizeof(float);
  if (lbm::overlap(g_pre, g_post, bytes))
    return fail(LBM_EINVAL, "gnn_forward: g_pre and g_post overlap");
  size_t need = forward_workspace_bytes(batch, nx, ny, n_rounds);
  if (!workspace || ws_bytes < need)
    return fail(LBM_EWORKSPACE, "gnn_forward: workspace needs %zu bytes", need);
  const size_t saved_need = gnn::saved_bytes(batch, nx, ny, n_rounds);
  if (saved && saved_bytes < saved_need)
    return fail(LBM_EWORKSPACE, "gnn_forward: saved buffer needs %zu bytes", saved_need);
  if (int rc = check_device()) return rc;
  return launch_forward(false, g_pre, g_post, batch, nx, ny, tau, 0.0f, params, n_rounds,
                        head_out, saved, workspace, nullptr, (hipStream_t)stream);
}

// lbm_step_gnn on a given scratch of forward_scratch(nx * ny) bytes or more.
static int step_gnn(const float *g_src, float *g_dst, int nx, int ny, float tau,
                    const float *params, int n_rounds, const lbm_fallback *fb, void *workspace,
                    hipStream_t s) {
  if (int rc = launch_forward(true, g_src, g_dst, 1, nx, ny, nullptr, tau, params, n_rounds,
                              nullptr, nullptr, workspace, fb, s))
    return rc;
  if (!fb) return LBM_OK;
  const ForwardScratch W = forward_scratch((long long)nx * ny);
  return launch_gate(g_src, g_dst, nx, ny, tau, 0, 0.0f, fb, at(workspace, W.pmass2),
                     at(workspace, W.ctrl), s);
}

static int check_step_gnn(const char *who, const float *g_src, float *g_dst, int nx, int ny,
                          float tau, const float *params, int n_rounds, const lbm_fallback *fb) {
  if (int rc = check_gnn_common(who, 1, nx, ny, params, n_rounds)) return rc;
  if (!g_src || !g_dst) return fail(LBM_EINVAL, "%s: null pointer", who);
  if (!(tau > 0.0f)) return fail(LBM_EINVAL, "%s: tau must be positive", who);
  size_t bytes = (size_t)9 * nx * ny * sizeof(float);
  if (lbm::overlap(g_src, g_dst, bytes))
    return fail(LBM_EINVAL, "%s: source and destination overlap", who);
  if (fb && (!fb->flags || !fb->mass))
    return fail(LBM_EINVAL, "%s: fallback needs flags and mass pointers", who);
  return LBM_OK;
}

extern "C" int lbm_step_gnn(const float *g_src, float *g_dst, int nx, int ny, float tau,
                            const float *params, int n_rounds, const lbm_fallback *fb,
                            void *workspace, size_t ws_bytes, void *stream) {
  if (int rc = check_step_gnn("lbm_step_gnn", g_src, g_dst, nx, ny, tau, params, n_rounds, fb))
    return rc;
  size_t need = step_workspace_bytes(nx, ny, n_rounds);
  if (!workspace || ws_bytes < need)
    return fail(LBM_EWORKSPACE, "lbm_step_gnn: workspace needs %zu bytes", need);
  if (int rc = check_device()) return rc;
  return step_gnn(g_src, g_dst, nx, ny, tau, params, n_rounds, fb, workspace,
                  (hipStream_t)stream);
}

// ------------------------------------------------- allocation-free step ---

// Scratch of lbm_step_gnn_noalloc: the forward scratch of the largest lattice
// it accepts, as a file-scope device array.  Every device the library runs
// on holds its own copy, at its own address.  In host code `scratch` names a
// host-side stand-in, not device memory: the device address of the current
// device's copy is looked up once with hipGetSymbolAddress and kept, and only
// that address is ever handed to kernels.
constexpr size_t kNoAllocBytes = forward_scratch(LBM_NOALLOC_MAX_NODES).total;
static_assert(kNoAllocBytes < (17u << 20), "the static scratch is documented as ~16.6 MiB");
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[64];  // device address of `scratch`, per device index

static int noalloc_scratch(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return fail(LBM_EDEVICE, "lbm_step_gnn_noalloc: hipGetDevice failed");
  if (dev < 0 || dev >= 64)
    return fail(LBM_EUNSUPPORTED, "lbm_step_gnn_noalloc: device index %d", dev);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LBM_EDEVICE, "lbm_step_gnn_noalloc: hipGetSymbolAddress: %s",
                  hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return LBM_OK;
}

extern "C" int lbm_step_gnn_noalloc(const float *g_src, float *g_dst, int nx, int ny, float tau,
                                    const float *params, int n_rounds, const lbm_fallback *fb,
                                    void *stream) {
  const char *who = "lbm_step_gnn_noalloc";
  if (int rc = check_step_gnn(who, g_src, g_dst, nx, ny, tau, params, n_rounds, fb)) return rc;
  if ((long long)nx * ny > LBM_NOALLOC_MAX_NODES)
    return fail(LBM_EINVAL, "%s: %d x %d lattice has more than the %d nodes its static scratch holds",
                who, nx, ny, LBM_NOALLOC_MAX_NODES);
  if (int rc = check_device()) return rc;
  void *ws = nullptr;
  if (int rc = noalloc_scratch(&ws)) return rc;
  // Everything the step reads from its scratch is written earlier in the same
  // step (the weight packing also zeroes the gate's arrival counts), so what
  // an earlier call left there does not matter.
  return step_gnn(g_src, g_dst, nx, ny, tau, params, n_rounds, fb, ws, (hipStream_t)stream);
}
