// The per-node corrected collision of the paper's Fig. 2 ("SimpleLBMGNN",
// Methodology, "GNN Architecture Details"): the distribution functions,
// density and velocity of one node go through two linear layers with ReLU and
// two heads, tau_adj (sigmoid scaled to [0.5, 1.5]) and the direct correction
// delta f, with no message passing between nodes.  With no neighbour
// dependence the whole network fuses into the pull step: one pass reads the
// nine populations of a node once and writes the corrected post-collision
// populations once, like the plain BGK step, with the network's BF16 MFMA
// work and the correction in registers.
//
// Sizes follow the corrected collision's encoder and head: 12 -> 64 -> 64
// (ReLU) -> 10.  The parameter blob is the zero-round layout:
//   W1[64][12] b1[64] W2[64][64] b2[64] Wh[10][64] bh[10] | mu[12] sigma[12] s_delta
// The weight fragments (gnn_prep_kernel), the gate's decision
// (gate_decide_last) and its fallback kernel are shared with the
// message-passing step; the collision epilogue is this
// file's own, with the same arithmetic except the hardware exp2 and
// reciprocal in the sigmoid and the relaxation rate.
#include "channel_common.hpp"
#include "gnn_common.hpp"
#include "lbm_common.hpp"

namespace gnn {

// Shared with gnn_kernels.hip.
int launch_prep(const float *params, int R, uint8_t *pack, unsigned *ctrl, hipStream_t s);

namespace simple {

using lbm::cx;
using lbm::cy;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

typedef short s16x2 __attribute__((ext_vector_type(2)));

// ReLU of eight accumulators, rounded to a BF16 B-operand fragment.  Rounding
// keeps the sign, so ReLU after rounding equals rounding after ReLU; on the
// packed BF16 bits ReLU is a signed 16-bit max with zero (negative values,
// -0 included, have the sign bit set), two values per instruction.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
  s16x2 h = __builtin_bit_cast(s16x2, v);
  h = __builtin_elementwise_max(h, s16x2{0, 0});
  return __builtin_bit_cast(uint32_t, h);
}

__device__ __forceinline__ u32x4 relu_frag(f32x4 lo, f32x4 hi) {
  u32x4 r = frag_from_acc(lo, hi);
  return u32x4{relu_bf16x2(r.x), relu_bf16x2(r.y), relu_bf16x2(r.z), relu_bf16x2(r.w)};
}

// Density deviation, density and velocity of a node, as lbm::node_moments
// (same sums, same order) but with the hardware reciprocal of rho (about
// 1 ulp) instead of an IEEE division.
__device__ __forceinline__ void moments(const float (&g)[9], float &drho, float &rho, float &u,
                                        float &v) {
  drho = ((g[0] + (g[1] + g[3])) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8]));
  const float jx = (g[1] - g[3]) + ((g[5] - g[7]) + (g[8] - g[6]));
  const float jy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
  rho = 1.0f + drho;
  const float inv = __builtin_amdgcn_rcpf(rho);
  u = jx * inv;
  v = jy * inv;
}

// Eq. 3 with the projected correction at one node, given its moments (the
// velocity without the force).  The sigmoid and the relaxation rate use the
// hardware exp2 and reciprocal (about 1 ulp each); z0 = 0 still gives
// tau_adj = 1 exactly (2^0 = 1, 1/2 = 0.5).  FORCED: under the channel's body
// force rho * gx, f^eq is taken at Guo's velocity and Guo's source is added at
// the effective rate omega = 1 / (tau tau_adj).
template <bool FORCED>
__device__ __forceinline__ void collide(float (&g)[9], const float (&z)[NOUT], float tau,
                                        float sdelta, float gx, float drho, float rho, float u,
                                        float v) {
  if constexpr (FORCED) u += 0.5f * gx;
  const float uu = u * u + v * v;
  constexpr float kLog2e = 1.4426950408889634f;
  float sig = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z[0] * kLog2e));
  float tau_adj = 0.5f + sig;
  float omega = __builtin_amdgcn_rcpf(tau * tau_adj);
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
  for (int i = 0; i < 9; ++i) {
    float relaxed = g[i] + omega * (lbm::geq_shifted<float>(i, drho, rho, u, v, uu) - g[i]);
    if constexpr (FORCED)
      relaxed += (1.0f - 0.5f * omega) * lbm::guo_source<float>(i, rho * gx, u, v);
    float df = z[1 + i] - m0 - float(cx(i)) * mx - float(cy(i)) * my;
    g[i] = relaxed + sdelta * df;
  }
}

// A wave takes 64 consecutive nodes of one lattice row (ChunkQueue), one
// node per lane for everything that is per node: the coalesced pull of the
// nine populations (kept in registers for the collision), the moments and the
// 12 normalised features (rounded to BF16 into the node's LDS slot), and the
// collision.  The network runs in between on MFMA, four column blocks of 16
// nodes with lane (n, q) = (node, channel group), two blocks at a time; each
// block reads its nodes' features and then writes their head outputs into the
// same slots.  Weight fragments and the (per channel group) bias fragments sit
// in LDS (one 48-byte slot per node keeps the block at 27 KB); each fragment
// read serves two blocks, which needs the registers of four blocks per CU
// instead of five and measured 8 % faster (the LDS reads of one block at a
// time moved ≈ 145 bytes per cycle per CU).
constexpr int kSlot = 12;   // dwords per node: 8 for the features, then 10 head outputs

constexpr int kBlocksPerCu = 4;   // resident blocks (LDS 27 KB, <= 128 registers)
constexpr int kBlocksPerCuSave = 3;   // the training forward, which also stores activations

// What a training forward keeps per node for the backward pass: the BF16
// operands the MFMAs consumed (features, both hidden layers, fragment order)
// and the FP32 head outputs; the layout of gnn_forward's saved buffer for
// zero rounds.
struct SimpleSave {
  uint16_t *x, *e1, *h0;
  float *z;
};

// WALLS (with PULL): the channel step, halfway bounce-back at rows 0 and
// ny - 1 and the body force rho * gx along x.
template <bool PULL, bool SAVE, bool WALLS>
__global__ __launch_bounds__(kThreads, SAVE ? kBlocksPerCuSave : kBlocksPerCu) void simple_step_kernel(
    const float *__restrict__ src, float *__restrict__ dst, int batch, int nx, int ny,
    const float *__restrict__ tau_arr, float tau_s, float gx, const uint8_t *__restrict__ pack,
    FragLayout F, float *__restrict__ head_out, Q80 *__restrict__ pmass,
    unsigned *__restrict__ pflag, SimpleSave sv, GateArgs gate, unsigned *__restrict__ chunkq) {
  __shared__ u32x4 w_s[14 * 64];   // W1 (4), W2 (8), Wh (2) fragments
  __shared__ f32x4 b_s[9 * 4];     // b1 (4), b2 (4), bh (1), per channel group
  __shared__ __attribute__((aligned(16))) uint32_t slot_s[kWaves][64 * kSlot];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  {
    const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
    const f32x4 *bias = (const f32x4 *)(pack + F.bias_off);
    for (int k = threadIdx.x; k < 14 * 64; k += kThreads) {
      int f = k >> 6, l = k & 63;
      int src_f = f < 4 ? F.W1 + f : (f < 12 ? F.W2 + (f - 4) : F.WH + (f - 12));
      w_s[k] = frags[(size_t)src_f * 64 + l];
    }
    // a bias fragment holds rows 4q..4q+3 for every node column: lane 16 q
    if (threadIdx.x < 9 * 4) {
      int b = threadIdx.x >> 2, g = threadIdx.x & 3;
      int src_b = b < 4 ? F.B1 + b : (b < 8 ? F.B2 + (b - 4) : F.BH);
      b_s[threadIdx.x] = bias[(size_t)src_b * 64 + 16 * g];
    }
  }
  const float *cst = (const float *)(pack + F.const_off);
  const float sdelta = cst[C_SDELTA];
  // normalisation (x - mu) / sigma as one FMA per feature: x * isg + nmi
  float isg[NFEAT], nmi[NFEAT];
#pragma unroll
  for (int k = 0; k < NFEAT; ++k) {
    isg[k] = 1.0f / cst[C_SIGMA + k];
    nmi[k] = -cst[C_MU + k] * isg[k];
  }
  __syncthreads();
  uint32_t *sw = slot_s[wave];
  Q80 mass_acc{0ull, 0ll};
  unsigned flag_acc = 0;

  const size_t row = (size_t)9 * nx;
  for (ChunkQueue cw(batch, nx, ny, kWaves, wave, chunkq); cw.more(); cw.next()) {
    const int xc = cw.xc, y = cw.y, b = cw.b;
    const float *lat = src + (size_t)b * ny * row;
    const int x = xc * 64 + lane;
    const bool valid = x < nx;
    const unsigned drawn = cw.draw();
    float gp[9];
    float drho, rho, u, v;  // kept for the collision
    {
      // rows y - 1, y, y + 1 (uniform) and columns x - 1, x, x + 1 (per lane)
      const int xv = valid ? x : nx - 1;
      const float *r0 = lat + (size_t)(y == 0 ? ny - 1 : y - 1) * row;
      const float *r1 = lat + (size_t)y * row;
      const float *r2 = lat + (size_t)(y == ny - 1 ? 0 : y + 1) * row;
      const int xs0 = xv == 0 ? nx - 1 : xv - 1, xs2 = xv == nx - 1 ? 0 : xv + 1;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        if constexpr (PULL) {
          // g_i(x, y) = post_i(x - c_ix, y - c_iy)
          const float *r = cy(i) > 0 ? r0 : (cy(i) < 0 ? r2 : r1);
          const int xsrc = cx(i) > 0 ? xs0 : (cx(i) < 0 ? xs2 : xv);
          if constexpr (WALLS) {
            // a population that would come through a wall is the reversed one
            // that left this node (the row is uniform over the wave)
            if ((cy(i) > 0 && y == 0) || (cy(i) < 0 && y == ny - 1))
              gp[i] = r1[(size_t)lbm::opp(i) * nx + xv];
            else
              gp[i] = r[(size_t)i * nx + xsrc];
          } else if (cx(i) == 0) {
            // no other chunk reads these lines (the shifted directions share
            // their edge lines with the neighbouring chunks): non-temporal,
            // -0.5 % (all nine non-temporal: +1.3 %)
            gp[i] = __builtin_nontemporal_load(r + (size_t)i * nx + xsrc);
          } else {
            gp[i] = r[(size_t)i * nx + xsrc];
          }
        } else {
          gp[i] = r1[(size_t)i * nx + xv];
        }
      }
    }
    {
      moments(gp, drho, rho, u, v);
      cw.take(drawn);
      const float uf = WALLS ? u + 0.5f * gx : u;  // Guo's velocity on the channel
      const float raw[NFEAT] = {gp[0], gp[1], gp[2], gp[3], gp[4], gp[5],
                                gp[6], gp[7], gp[8], drho, uf,    v};
      float ft[NFEAT];
#pragma unroll
      for (int k = 0; k < NFEAT; ++k) ft[k] = fmaf(raw[k], isg[k], nmi[k]);
      u32x4 *o = (u32x4 *)(sw + lane * kSlot);
      o[0] = u32x4{pack_bf16(ft[0], ft[1]), pack_bf16(ft[2], ft[3]), pack_bf16(ft[4], ft[5]),
                   pack_bf16(ft[6], ft[7])};
      o[1] = u32x4{pack_bf16(ft[8], ft[9]), pack_bf16(ft[10], ft[11]), 0u, 0u};
    }
    wave_lds_sync();
    // Two column blocks of 16 nodes at a time: each weight and bias fragment
    // read from LDS serves both (half the LDS reads of one block at a time).
#pragma unroll 2
    for (int pair = 0; pair < 2; ++pair) {
      int wo = lane;
      asm volatile("" : "+v"(wo));
      const u32x4 *w = w_s + wo;
      const f32x4 *bs = b_s + q;
      uint32_t *slot[2];
      u32x4 xb[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        slot[h] = sw + (16 * (2 * pair + h) + n) * kSlot;
        xb[h] = q < 2 ? *(const u32x4 *)(slot[h] + 4 * q) : u32x4{0u, 0u, 0u, 0u};
      }
      f32x4 a[2][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const u32x4 wt = w[t * 64];
        const f32x4 bt = bs[t * 4];
#pragma unroll
        for (int h = 0; h < 2; ++h) a[h][t] = mfma(wt, xb[h], bt);
      }
      u32x4 e1[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        e1[h][0] = relu_frag(a[h][0], a[h][1]);
        e1[h][1] = relu_frag(a[h][2], a[h][3]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const u32x4 w0 = w[(4 + 2 * t) * 64], w1 = w[(5 + 2 * t) * 64];
        const f32x4 bt = bs[(4 + t) * 4];
#pragma unroll
        for (int h = 0; h < 2; ++h) a[h][t] = mfma(w1, e1[h][1], mfma(w0, e1[h][0], bt));
      }
      u32x4 hb[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        hb[h][0] = relu_frag(a[h][0], a[h][1]);
        hb[h][1] = relu_frag(a[h][2], a[h][3]);
      }
      if constexpr (SAVE) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int xs = xc * 64 + 16 * (2 * pair + h) + n;
          if (xs < nx) {
            const size_t node = ((size_t)b * ny + y) * nx + xs;
            if (q < 2) ((u32x4 *)(sv.x + node * 16))[q] = xb[h];
            u32x4 *de = (u32x4 *)(sv.e1 + node * HID);
            de[q] = e1[h][0];
            de[4 + q] = e1[h][1];
            u32x4 *dh = (u32x4 *)(sv.h0 + node * HID);
            dh[q] = hb[h][0];
            dh[4 + q] = hb[h][1];
          }
        }
      }
      const u32x4 w12 = w[12 * 64], w13 = w[13 * 64];
      const f32x4 b8 = bs[8 * 4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 z = mfma(w13, hb[h][1], mfma(w12, hb[h][0], b8));
        // the features of these 16 nodes are consumed (z depends on them):
        // their slots take the head outputs, rows 4q..4q+3
        if (q < 2) *(f32x4 *)(slot[h] + 4 * q) = z;
        else if (q == 2) *(float2 *)(slot[h] + 8) = float2{z.x, z.y};
      }
    }
    wave_lds_sync();
    if (valid) {
      float z[NOUT];
      {
        const f32x4 *zs = (const f32x4 *)(sw + lane * kSlot);
        const f32x4 z0 = zs[0], z1 = zs[1], z2 = zs[2];
        const float zz[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w, z2.x, z2.y, z2.z, z2.w};
#pragma unroll
        for (int k = 0; k < NOUT; ++k) z[k] = zz[k];
      }
      const float tau = tau_arr ? tau_arr[b] : tau_s;  // b < batch while cw.more()
      collide<WALLS>(gp, z, tau, sdelta, gx, drho, rho, u, v);
      float *d = dst + (size_t)b * ny * row + (size_t)y * row + x;
      // node mass in FP32 (rounding ~1e-9 per node, ~1e-13 of the lattice
      // mass), accumulated over the nodes in exact fixed point (a total that
      // does not depend on which wave took which chunk).  A population is negative
      // or not finite exactly when the smallest f_i is below zero or the sum
      // is not finite (an infinity or NaN anywhere reaches the sum; the
      // minimum skips NaN).
      float msum = 0.0f, fmin = INFINITY;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        __builtin_nontemporal_store(gp[i], d + (size_t)i * nx);
        fmin = fminf(fmin, gp[i] + lbm::wgt<float>(i));
        msum += gp[i];
      }
      const unsigned bad = (fmin >= 0.0f && fabsf(msum) < INFINITY) ? 0u : 1u;
      mass_acc = q80_add_f32(mass_acc, msum);
      flag_acc |= bad;
      if (head_out) {
        const size_t node = ((size_t)b * ny + y) * nx + x;
        for (int k = 0; k < NOUT; ++k) head_out[node * NOUT + k] = z[k];
      }
      if constexpr (SAVE) {
        const size_t node = ((size_t)b * ny + y) * nx + x;
#pragma unroll
        for (int k = 0; k < NOUT; ++k) sv.z[node * 12 + k] = z[k];
      }
    }
    wave_lds_sync();
  }

  // every wave is done with its slots: the reduction reuses them
  __syncthreads();
  Q80 *red_m = (Q80 *)&slot_s[0][0];
  unsigned *red_f = &slot_s[0][0] + 4 * kThreads;
  static_assert(5 * kThreads <= kWaves * 64 * kSlot, "reduction fits in the slots");
  red_m[threadIdx.x] = mass_acc;
  red_f[threadIdx.x] = flag_acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red_m[threadIdx.x] = q80_add(red_m[threadIdx.x], red_m[threadIdx.x + s]);
      red_f[threadIdx.x] |= red_f[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pmass[blockIdx.x] = red_m[0];
    pflag[blockIdx.x] = red_f[0];
  }
  if constexpr (PULL) {
    if (gate.ctrl)
      gate_decide_last<kThreads>(gate, pmass, pflag, (int)gridDim.x, (double)nx * ny, red_m,
                                 red_f);
  }
}

}  // namespace simple

// The gate's fallback kernel, shared with the message-passing step (gnn_kernels.hip).
int launch_gate(const float *g_src, float *g_dst, int nx, int ny, float tau, int walls,
                float gx, const lbm_fallback *fb, void *pmass2, void *ctrl, hipStream_t s);

}  // namespace gnn

using namespace gnn;
using lbm::check_device;
using lbm::fail;
using lbm::launch_check;

static inline void *at_(void *base, size_t off) { return (uint8_t *)base + off; }

static int simple_device_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      v <= 0)
    return 256;
  return v;
}

// pull: the fused step (else the forward of pre-collision states); walls: the
// channel step (with pull), body force rho * gx along x.
static int launch_simple(bool pull, bool walls, float gx, const float *src, float *dst,
                         int batch, int nx, int ny, const float *tau_arr, float tau,
                         const float *params, float *head_out, void *saved, void *ws,
                         const lbm_fallback *fb, hipStream_t s) {
  const FragLayout F = frag_layout(0);
  const SimpleScratch W = simple_scratch();
  uint8_t *pack = (uint8_t *)at_(ws, W.pack);
  unsigned *ctrl = (unsigned *)at_(ws, W.ctrl);
  if (int rc = launch_prep(params, 0, pack, ctrl, s)) return rc;
  const long long chunks = (long long)batch * ny * ((nx + 63) / 64);
  long long blocks = (chunks + simple::kWaves - 1) / simple::kWaves;
  // the resident blocks; their waves draw the chunks from a counter
  long long cap = (long long)simple_device_cus() *
                  (saved && !pull ? simple::kBlocksPerCuSave : simple::kBlocksPerCu);
  if (cap > kMaxGnnBlocks) cap = kMaxGnnBlocks;
  const int nb = (int)(blocks < cap ? blocks : cap);
  Q80 *pm = (Q80 *)at_(ws, W.pmass);
  unsigned *pf = (unsigned *)at_(ws, W.pflag);
  GateArgs gate{};
  if (fb && pull) gate = GateArgs{ctrl, fb->drift_threshold, fb->flags, fb->n_fallback, fb->mass};
  simple::SimpleSave sv{};
  if (saved) {
    const SavedLayout SL = saved_layout((long long)batch * nx * ny, 0);
    sv.x = (uint16_t *)at_(saved, SL.x);
    sv.e1 = (uint16_t *)at_(saved, SL.e1);
    sv.h0 = (uint16_t *)at_(saved, SL.h);
    sv.z = (float *)at_(saved, SL.z);
  }
  if (pull && walls)
    hipLaunchKernelGGL((simple::simple_step_kernel<true, false, true>), dim3(nb),
                       dim3(simple::kThreads), 0, s, src, dst, batch, nx, ny, tau_arr, tau, gx,
                       pack, F, head_out, pm, pf, sv, gate, ctrl + kCtrlChunkQueue);
  else if (pull)
    hipLaunchKernelGGL((simple::simple_step_kernel<true, false, false>), dim3(nb),
                       dim3(simple::kThreads), 0, s, src, dst, batch, nx, ny, tau_arr, tau, 0.0f,
                       pack, F, head_out, pm, pf, sv, gate, ctrl + kCtrlChunkQueue);
  else if (saved)
    hipLaunchKernelGGL((simple::simple_step_kernel<false, true, false>), dim3(nb),
                       dim3(simple::kThreads), 0, s, src, dst, batch, nx, ny, tau_arr, tau, 0.0f,
                       pack, F, head_out, pm, pf, sv, gate, ctrl + kCtrlChunkQueue);
  else
    hipLaunchKernelGGL((simple::simple_step_kernel<false, false, false>), dim3(nb),
                       dim3(simple::kThreads), 0, s, src, dst, batch, nx, ny, tau_arr, tau, 0.0f,
                       pack, F, head_out, pm, pf, sv, gate, ctrl + kCtrlChunkQueue);
  return launch_check("simple_step_kernel");
}

static int check_simple(const char *who, int batch, int nx, int ny, const float *params) {
  if (!params) return fail(LBM_EINVAL, "%s: null parameters", who);
  if (batch < 1 || !lbm::lattice_ok(nx, ny) || (long long)batch * nx * ny >= (1LL << 31))
    return fail(LBM_EINVAL, "%s: bad sizes batch %d, %d x %d", who, batch, nx, ny);
  return LBM_OK;
}

extern "C" int simple_forward(const float *g_pre, float *g_post, int batch, int nx, int ny,
                              const float *tau, const float *params, float *head_out,
                              void *saved, size_t saved_bytes, void *workspace,
                              size_t ws_bytes, void *stream) {
  if (int rc = check_simple("simple_forward", batch, nx, ny, params)) return rc;
  if (!g_pre || !g_post || !tau) return fail(LBM_EINVAL, "simple_forward: null pointer");
  if (lbm::overlap(g_pre, g_post, (size_t)batch * 9 * nx * ny * sizeof(float)))
    return fail(LBM_EINVAL, "simple_forward: g_pre and g_post overlap");
  if (!workspace || ws_bytes < simple_scratch().total)
    return fail(LBM_EWORKSPACE, "simple_forward: workspace needs %zu bytes",
                simple_scratch().total);
  const size_t saved_need = gnn::saved_bytes(batch, nx, ny, 0);
  if (saved && saved_bytes < saved_need)
    return fail(LBM_EWORKSPACE, "simple_forward: saved buffer needs %zu bytes", saved_need);
  if (int rc = check_device()) return rc;
  return launch_simple(false, false, 0.0f, g_pre, g_post, batch, nx, ny, tau, 0.0f, params,
                       head_out, saved, workspace, nullptr, (hipStream_t)stream);
}

// The fused step, periodic (walls = 0) or the channel (walls = 1, force gx).
static int step_simple(const char *who, const float *g_src, float *g_dst, int nx, int ny,
                       float tau, bool walls, float gx, const float *params,
                       const lbm_fallback *fb, void *workspace, size_t ws_bytes, void *stream) {
  if (int rc = check_simple(who, 1, nx, ny, params)) return rc;
  if (!g_src || !g_dst) return fail(LBM_EINVAL, "%s: null pointer", who);
  if (!(tau > 0.0f)) return fail(LBM_EINVAL, "%s: tau must be positive", who);
  if (walls && !(gx == gx && fabsf(gx) < INFINITY))
    return fail(LBM_EINVAL, "%s: force must be finite", who);
  if (lbm::overlap(g_src, g_dst, (size_t)9 * nx * ny * sizeof(float)))
    return fail(LBM_EINVAL, "%s: source and destination overlap", who);
  if (fb && (!fb->flags || !fb->mass))
    return fail(LBM_EINVAL, "%s: fallback needs flags and mass pointers", who);
  if (!workspace || ws_bytes < simple_scratch().total)
    return fail(LBM_EWORKSPACE, "%s: workspace needs %zu bytes", who, simple_scratch().total);
  if (int rc = check_device()) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (int rc = launch_simple(true, walls, gx, g_src, g_dst, 1, nx, ny, nullptr, tau, params,
                             nullptr, nullptr, workspace, fb, s))
    return rc;
  if (!fb) return LBM_OK;
  const SimpleScratch W = simple_scratch();
  return launch_gate(g_src, g_dst, nx, ny, tau, walls ? 1 : 0, gx, fb, at_(workspace, W.pmass2),
                     at_(workspace, W.ctrl), s);
}

extern "C" int lbm_step_simple(const float *g_src, float *g_dst, int nx, int ny, float tau,
                               const float *params, const lbm_fallback *fb, void *workspace,
                               size_t ws_bytes, void *stream) {
  return step_simple("lbm_step_simple", g_src, g_dst, nx, ny, tau, false, 0.0f, params, fb,
                     workspace, ws_bytes, stream);
}

extern "C" int lbm_step_simple_channel(const float *g_src, float *g_dst, int nx, int ny,
                                       float tau, float gx, const float *params,
                                       const lbm_fallback *fb, void *workspace,
                                       size_t ws_bytes, void *stream) {
  return step_simple("lbm_step_simple_channel", g_src, g_dst, nx, ny, tau, true, gx, params, fb,
                     workspace, ws_bytes, stream);
}
