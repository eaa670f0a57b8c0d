// Device building blocks of the GNN-corrected collision on gfx950:
// BF16 fragments for v_mfma_f32_16x16x32_bf16, the activation functions and
// the packed weight-fragment buffer written by gnn_prep_kernel.
//
// Orientation.  Every dense layer is computed transposed, out^T = W in^T:
// the 16x16 MFMA tile has output channels as rows (M) and nodes as columns
// (N), and the contraction runs over input channels (K).  A wave therefore
// processes 16 nodes at a time and holds, after an MFMA, in lane l = 16 q + n
// (n = node 0..15, q = 0..3) the outputs of channels 16 t + 4 q + e (e = 0..3)
// of row tile t.  The B operand of a 16x16x32 step holds, in the same lane,
// 8 input values of node n.  Choosing the 8 values of k-step s to be the
// outputs of row tiles 2s and 2s+1 of the previous layer, i.e. input channel
//     c(s, q, j) = 16 (2 s + j / 4) + 4 q + j % 4,     j = 0..7,
// makes a layer's FP32 accumulators, rounded to BF16, exactly the next
// layer's B operand: layers chain in registers with no data movement.  The
// weights (A operand) are stored with their input columns permuted the same
// way.  Node states stored in memory use this "fragment order": position
// p = 32 s + 8 q + j of a node's 64 values holds channel c(s, q, j).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gnn_layout.hpp"

namespace gnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Input channel (natural index) behind element j of k-step s in lane group q.
__host__ __device__ constexpr int frag_channel(int s, int q, int j) {
  return 16 * (2 * s + j / 4) + 4 * q + (j % 4);
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Two FP32 values rounded to nearest-even BF16, packed low/high
// (v_cvt_pk_bf16_f32).
// Two floats rounded to nearest-even BF16, lo in bits 0..15: one
// v_cvt_pk_bf16_f32 with both operands.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) {
  return __uint_as_float(bits16 << 16);
}

// B-operand fragment of k-step s from the FP32 accumulators of row tiles
// 2s and 2s+1.
__device__ __forceinline__ u32x4 frag_from_acc(f32x4 lo, f32x4 hi) {
  u32x4 r;
  r.x = pack_bf16(lo.x, lo.y);
  r.y = pack_bf16(lo.z, lo.w);
  r.z = pack_bf16(hi.x, hi.y);
  r.w = pack_bf16(hi.z, hi.w);
  return r;
}

// BF16 bits of a small integer in {-1, 0, 1}.
__host__ __device__ constexpr uint32_t bf16_unit(int v) {
  return v == 0 ? 0u : (v > 0 ? 0x3f80u : 0xbf80u);
}

// GELU, tanh form: 0.5 x (1 + tanh(k0 (x + k1 x^3))) = x / (1 + 2^t) with
// t = -2 k0 log2(e) (x + k1 x^3).  One hardware exp2 and one reciprocal.
constexpr float kGeluA = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
constexpr float kGeluB = kGeluA * 0.044715f;
constexpr float kLn2 = 0.6931471805599453f;

__device__ __forceinline__ float gelu(float x) {
  float t = x * __builtin_fmaf(x * x, kGeluB, kGeluA);
  float e = __builtin_amdgcn_exp2f(t);
  return x * __builtin_amdgcn_rcpf(1.0f + e);
}

// d GELU / dx = s - x s (1 - s) ln2 (A + 3 B x^2), s = 1 / (1 + 2^t),
// evaluated as s (1 - w + w s) with w = x ln2 (A + 3 B x^2) and ln2 folded
// into the constants: 11 VALU instructions, two of them transcendental.
constexpr float kGeluDA = kGeluA * kLn2;
constexpr float kGeluDB = 3.0f * kGeluB * kLn2;
__device__ __forceinline__ float gelu_grad(float x) {
  float x2 = x * x;
  float t = x * __builtin_fmaf(x2, kGeluB, kGeluA);
  float s = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
  float w = x * __builtin_fmaf(x2, kGeluDB, kGeluDA);
  return s * __builtin_fmaf(w, s, 1.0f - w);
}

__device__ __forceinline__ f32x4 gelu4(f32x4 v) {
  return f32x4{gelu(v.x), gelu(v.y), gelu(v.z), gelu(v.w)};
}

// ------------------------------------------------------------------------
// Packed weights.  gnn_prep_kernel converts the FP32 blob into BF16
// A-operand fragments (1 KiB each: 64 lanes x 16 B) and FP32 bias fragments
// in accumulator layout (1 KiB each: 64 lanes x 4 floats).  Forward
// fragments first; the transposed weights used by the backward pass follow.
// ------------------------------------------------------------------------
struct FragLayout {
  // A-operand fragments, index of (tile, k-step) 0
  int W1, W2, WA[MAX_ROUNDS], WB[MAX_ROUNDS], WC[MAX_ROUNDS], WN[MAX_ROUNDS], WH;
  // transposed weights for the backward pass
  int W2T, WAT[MAX_ROUNDS], WBT[MAX_ROUNDS], WNT[MAX_ROUNDS], WHT;
  int nfrag;
  // bias fragments
  int B1, B2, BE[MAX_ROUNDS], BN[MAX_ROUNDS], BH;
  int nbias;
  // byte offsets inside the packed buffer
  size_t frag_off, bias_off, const_off, total;
};

__host__ __device__ inline FragLayout frag_layout(int R) {
  FragLayout F{};
  int f = 0;
  F.W1 = f; f += 4;          // 4 row tiles x 1 k-step (K = 12 padded to 32)
  F.W2 = f; f += 8;          // 4 x 2
  for (int r = 0; r < R; ++r) {
    F.WA[r] = f; f += 8;     // 4 x 2   receiver part of the edge layer
    F.WB[r] = f; f += 8;     // 4 x 2   sender part
    F.WC[r] = f; f += 4;     // 4 x 1   edge-direction part (K = 2 padded)
    F.WN[r] = f; f += 16;    // 4 x 4   node update, K = 128
  }
  F.WH = f; f += 2;          // 1 x 2   head (10 rows padded to 16)
  F.W2T = f; f += 8;         // W2^T       4 x 2
  for (int r = 0; r < R; ++r) {
    F.WAT[r] = f; f += 8;    // Wa^T       4 x 2
    F.WBT[r] = f; f += 8;    // Wb^T       4 x 2
    F.WNT[r] = f; f += 16;   // Wn^T       8 x 2 (128 rows)
  }
  F.WHT = f; f += 4;         // Wh^T       4 x 1 (K = 10 padded to 32)
  F.nfrag = f;
  int b = 0;
  F.B1 = b; b += 4;
  F.B2 = b; b += 4;
  for (int r = 0; r < R; ++r) {
    F.BE[r] = b; b += 4;
    F.BN[r] = b; b += 4;
  }
  F.BH = b; b += 1;
  F.nbias = b;
  F.frag_off = 0;
  F.bias_off = (size_t)F.nfrag * 1024;
  F.const_off = F.bias_off + (size_t)F.nbias * 1024;
  F.total = align256(F.const_off + 32 * sizeof(float));
  return F;
}

// Constants after the bias fragments (FP32): mu[12], sigma[12], s_delta.
constexpr int C_MU = 0, C_SIGMA = 12, C_SDELTA = 24;

__device__ __forceinline__ u32x4 load_frag(const u32x4 *__restrict__ frags, int f, int lane) {
  return frags[(size_t)f * 64 + lane];
}
__device__ __forceinline__ f32x4 load_bias(const f32x4 *__restrict__ bias, int b, int lane) {
  return bias[(size_t)b * 64 + lane];
}

// Packs the FP32 blob into `pack` (frag_layout(R).total bytes) on stream s.
int launch_prep(const float *params, int R, uint8_t *pack, unsigned *ctrl, hipStream_t s);

// Chunks of 64 consecutive nodes of a lattice row, chunk c = (b ny + y) cxn
// + xc over `batch` lattices of nx x ny (batch nx ny < 2^31 keeps every index
// in int), handed out to the waves dynamically, so that waves that are
// issued first (the hardware favours the oldest workgroup of a CU) take more
// chunks and all of them finish together; with a fixed share per wave the
// last waves ran on alone for a third of the kernel.  The chunks are split
// into kQueueParts contiguous parts, part p served by the workgroups
// b = p (mod parts) (consecutive workgroups go to different XCDs, so each
// part stays on one), each with its own counter: one counter for the whole
// grid serialised the atomics.  A wave works through batches of kQueueBatch
// consecutive chunks: its first batch by its index in the part, every later
// one from the part's counter, drawn by lane 0 in the first chunk of the
// previous batch, so the atomic's latency hides behind that chunk's loads.
// Every member is wave-uniform.  No result depends on which wave takes a
// chunk.
constexpr int kQueueParts = 8;
constexpr int kQueueBatch = 4;
constexpr int kQueueStride = 32;  // words between two part counters (128 bytes)

struct ChunkQueue {
  int c, xc, y, b;  // current chunk, c >= nchunks when done
  int cxn, ny, nchunks;
  int base, len, cur, end, first_dyn;
  unsigned *ctr;
  int nxt;     // first chunk (in the part) of the next batch, once taken
  bool fresh;  // the current chunk starts its batch: its draw is to be issued and taken
  __device__ __forceinline__ ChunkQueue(int batch, int nx, int ny_, int waves_per_block,
                                        int wave, unsigned *counters) {
    const int w = __builtin_amdgcn_readfirstlane(wave);
    cxn = (nx + 63) >> 6;
    ny = ny_;
    nchunks = batch * ny * cxn;
    const int G = (int)gridDim.x, parts = G < kQueueParts ? G : kQueueParts;
    const int p = (int)blockIdx.x % parts;
    const int L = (nchunks + parts - 1) / parts;
    base = p * L;
    len = nchunks - base < L ? nchunks - base : L;
    const int part_waves = ((G - 1 - p) / parts + 1) * waves_per_block;
    first_dyn = part_waves * kQueueBatch;
    ctr = counters + p * kQueueStride;
    nxt = len;
    cur = ((int)blockIdx.x / parts * waves_per_block + w) * kQueueBatch;
    begin_batch();
  }
  __device__ __forceinline__ void at(int local) {
    c = base + local;
    xc = c % cxn;
    y = (c / cxn) % ny;
    b = c / cxn / ny;
  }
  __device__ __forceinline__ void begin_batch() {
    if (cur >= len) {
      c = nchunks;
      return;
    }
    end = cur + kQueueBatch < len ? cur + kQueueBatch : len;
    at(cur);
    fresh = true;
  }
  // In the first chunk of a batch, lane 0 draws the next batch: draw() before
  // the chunk's loads, take() once they have been waited for (which waited for
  // the draw too).  The draw passes from one to the other in a register local
  // to the chunk, so no register still waiting for the atomic is carried
  // around the loop: such a register is copied at the loop's end, and the copy
  // waited for every memory operation, the chunk's fresh stores included.
  __device__ __forceinline__ unsigned draw() const {
    unsigned d = 0;
    if (fresh && (threadIdx.x & 63) == 0) {
      // an address the compiler cannot prove wave-uniform: otherwise it makes
      // the one-lane atomic wave-wide and waits for its result at once
      int z = 0;
      asm volatile("" : "+v"(z));
      d = atomicAdd(ctr + z, (unsigned)kQueueBatch);
    }
    return d;
  }
  __device__ __forceinline__ void take(unsigned d) {
    if (fresh) {
      nxt = first_dyn + (int)__builtin_amdgcn_readfirstlane(d);
      fresh = false;
    }
  }
  __device__ __forceinline__ bool more() const { return c < nchunks; }
  __device__ __forceinline__ void next() {
    if (++cur < end) {
      at(cur);
      return;
    }
    cur = nxt;
    begin_batch();
  }
};

// Makes the LDS writes of this wave visible to all of its lanes before the
// reads that follow (LDS staging private to one wave).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ gate ---

// The per-step fallback gate, as seen by the kernel that produces the
// corrected step's per-workgroup FP64 mass and flag partials.  Control words
// (in the caller's workspace): ctrl[0] = the step's decision, ctrl[1] =
// workgroups of the producing kernel done, ctrl[2] = workgroups of the
// fallback kernel done.  gnn_prep_kernel, which starts every step, zeroes
// the two counts, the tile counters of the message-passing rounds,
// ctrl[kCtrlTileQueue + r], and the chunk counters of the encoder or of the
// fused per-node step, ctrl[kCtrlChunkQueue + 32 p].  arrive == NULL means the step runs without the
// gate.
constexpr int kCtrlTileQueue = 4;
constexpr int kCtrlChunkQueue = 32;  // kQueueParts counters, 128 bytes apart
static_assert(kCtrlTileQueue + MAX_ROUNDS <= kCtrlChunkQueue, "control words");
static_assert(kCtrlChunkQueue + kQueueParts * kQueueStride <= kCtrlWords, "control words fit their bytes");
struct GateArgs {
  unsigned *ctrl;        // control words above, or NULL (no gate)
  double threshold;      // relative mass drift allowed per step
  unsigned *flags;       // OR-ed: 1 = negative / non-finite population, 2 = drift
  unsigned *n_fallback;  // steps that fell back, or NULL
  double *mass;          // total mass of the previous state (FP64), in/out
};

// Mass partials in exact fixed point: a signed 128-bit integer in units of
// 2^-80 (hi * 2^64 + lo).  Integer addition is associative, so a total does
// not depend on the order its terms are added in, which lets the last round
// hand out tiles to whichever workgroup is free and still take the same gate
// decision and record the same mass for the same state.  Each term is an
// FP64 sum of a few FP32 populations; it is clamped to +-256 (a node whose
// populations reach that has long failed the drift check; the clamp keeps
// 2^27 terms far from overflow: 2^27 * 2^8 * 2^80 = 2^115) and truncated to
// the grid (error below 2^-80 per term), NaN counting as 0 (the population
// check flags it).
struct Q80 {
  unsigned long long lo;
  long long hi;
};

__device__ __forceinline__ Q80 q80_add(Q80 a, Q80 b) {
  Q80 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

__device__ __forceinline__ Q80 q80_of(double v) {
  if (!(v == v)) v = 0.0;
  v = fmin(fmax(v, -256.0), 256.0);
  const double sc = v * 65536.0;  // exact: a power of two
  const double h = floor(sc);
  const double r = sc - h;        // exact, in [0, 1)
  Q80 q;
  q.hi = (long long)h;
  q.lo = (unsigned long long)(r * 18446744073709551616.0);  // r * 2^64 < 2^64
  return q;
}

// Adds an FP32 value, rounded to the nearest multiple of 2^-40 (clamped
// to +-256, as above), with full-rate FP32 and integer instructions only:
// v 2^16 = h + r exactly (h integer, 0 <= r < 1), then r 2^24 is rounded to an
// integer u, and the term is (h 2^24 + u) 2^-40 = (h 2^64 + u 2^40) 2^-80.
__device__ __forceinline__ Q80 q80_add_f32(Q80 a, float v) {
  v = __builtin_amdgcn_fmed3f(v, -256.0f, 256.0f);
  const float sc = v * 65536.0f;                 // exact, |sc| <= 2^24
  const float h = floorf(sc);
  const float r = sc - h;                        // exact, in [0, 1)
  const unsigned u = (unsigned)(r * 16777216.0f + 0.5f);  // <= 2^24 (2^24: a carry)
  const int hi = (int)h + (int)(u >> 24);
  // term = hi * 2^64 + (u mod 2^24) * 2^40 in 128 bits
  const unsigned long long lo = (unsigned long long)(u & 0xFFFFFFu) << 40;
  Q80 out;
  out.lo = a.lo + lo;
  out.hi = a.hi + (long long)hi + (out.lo < a.lo ? 1 : 0);
  return out;
}

// The value rounded to FP64 (the same integer always gives the same double).
__device__ __forceinline__ double q80_value(Q80 q) {
  return (double)q.hi * (1.0 / 65536.0) + (double)q.lo * 0x1p-80;
}

// Partial sums of either kind, added and read out in the gate below.
__device__ __forceinline__ double part_add(double a, double b) { return a + b; }
__device__ __forceinline__ Q80 part_add(Q80 a, Q80 b) { return q80_add(a, b); }
__device__ __forceinline__ double part_value(double a) { return a; }
__device__ __forceinline__ double part_value(Q80 a) { return q80_value(a); }
template <typename P>
__device__ __forceinline__ P part_zero() { return P{}; }

// Called by all kThreads threads of every workgroup of the producing kernel,
// after its thread 0 stored the workgroup's partials.  The workgroup that
// finishes last sums every partial in index order (a fixed order: the same
// decision for the same state) and decides: bit 1 = a negative or non-finite
// population, bit 2 = relative change of total mass not <= threshold.  A
// kept step records its new mass here; a tripped one records the flags and
// the fallback count, and the fallback kernel then writes the mass of what it
// stored.  sm and sf are shared scratch of kThreads entries each; every
// thread takes part in the barriers, so no thread may have left before.
template <int kThreads, typename P>
__device__ void gate_decide_last(const GateArgs &g, const P *pmass, const unsigned *pflag,
                                 int nparts, double nodes, P *sm, unsigned *sf) {
  if (threadIdx.x == 0) {
    __threadfence();  // this workgroup's partials before its arrival
    const unsigned done = atomicAdd(&g.ctrl[1], 1u);
    sf[0] = done == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  const bool last = sf[0] != 0u;
  __syncthreads();
  if (!last) return;
  __threadfence();  // every other workgroup's partials are visible
  P m = part_zero<P>();
  unsigned f = 0;
  for (int k = threadIdx.x; k < nparts; k += kThreads) {
    m = part_add(m, pmass[k]);
    f |= pflag[k];
  }
  sm[threadIdx.x] = m;
  sf[threadIdx.x] = f;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[threadIdx.x] = part_add(sm[threadIdx.x], sm[threadIdx.x + s]);
      sf[threadIdx.x] |= sf[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mnew = nodes + part_value(sm[0]);
    const double mold = *g.mass;
    unsigned fl = sf[0] ? 1u : 0u;
    const double rel = fabs(mnew - mold) / mold;
    if (!(rel <= g.threshold)) fl |= 2u;
    g.ctrl[0] = fl;
    if (fl) {
      *g.flags |= fl;
      if (g.n_fallback) *g.n_fallback += 1u;
    } else {
      *g.mass = mnew;
    }
  }
}

}  // namespace gnn
