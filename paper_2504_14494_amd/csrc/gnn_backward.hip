// Backward pass of the GNN-corrected collision and the pieces of one
// training step (paper: Training Methodology, loss of Eq. 4): gradient of a
// scalar loss with respect to every trainable parameter, the MSE loss and an
// Adam update.  n_rounds >= 1 is the message-passing network (GELU);
// n_rounds = 0 the per-node network of Fig. 2 (ReLU): head, then encoder.
//
// The forward saved, per node, the BF16 values the MFMAs consumed: features
// x, first encoder layer e1, node states h_0..h_R and summed messages a_1..a_R,
// plus the FP32 head outputs z.  BF16 rounding is differentiated as the
// identity.  Pre-activations are recomputed from those values.
//
// Per round r (h = h_r, h' = h_{r+1}, a = a_{r+1}), with p = Wn [h; a] + bn,
// q_{n,d} = Wa h_n + Wb h_{n+e_d} + Wc e_d + be and G = dL/dh':
//   dp = G . gelu'(p)                       dWn += dp [h; a]^T, dbn += dp
//   [dh ; da] = Wn^T dp
//   dq_{n,d} = da_n . gelu'(q_{n,d})        T_n = sum_d dq_{n,d}
//   dWa += T_n h_n^T, dbe += T_n, dWc += sum_d dq_{n,d} e_d^T, dh_n += Wa^T T_n
//   S_m = sum_d dq_{m-e_d,d}                dWb += S_m h_m^T,  dh_m += Wb^T S_m
// The sender sum S_m is a gather: dq is stored per edge (BF16) by the
// receiver-side kernel and read back by the sender-side kernel, so no
// gradient is ever scattered.
//
// Weight gradients are MFMA products with the node index as contraction
// dimension.  Each wave stages 32 nodes' gradient rows and activation rows
// transposed (channel-major, BF16) in its own LDS, accumulates dW over all
// the nodes it visits, and writes one FP32 partial per wave; a last kernel
// sums the partials of the fixed grid in a fixed order, so the gradient is
// bitwise reproducible.
#include "gnn_common.hpp"
#include "lbm_common.hpp"

namespace gnn {

using lbm::cx;
using lbm::cy;

constexpr int kBT = 256;            // threads per block
constexpr int kPitch = 40;          // BF16 per staged row: 32 nodes + padding

// ------------------------------------------------------------ helpers ---

struct Pos {
  int b, y, x;          // x clamped into the lattice for loads
  bool valid;
  size_t node;
};

__device__ __forceinline__ Pos group_pos(long long grp, long long ngroups, int n, int nx, int ny,
                                         long long gxn) {
  Pos P;
  bool in = grp < ngroups;
  long long g = in ? grp : 0;
  int xg = (int)(g % gxn);
  long long by = g / gxn;
  P.y = (int)(by % ny);
  P.b = (int)(by / ny);
  int x = xg * 16 + n;
  P.valid = in && x < nx;
  P.x = x < nx ? x : x % nx;
  P.node = ((size_t)P.b * ny + P.y) * nx + P.x;
  return P;
}

// FP32 per-node vectors in accumulator order: lane (n, q) owns the 64 bytes
// at q * 16 floats (row tiles t = 0..3, 4 values each).
__device__ __forceinline__ void load_acc(const float *buf, size_t node, int q, f32x4 (&v)[4]) {
  const f32x4 *p = (const f32x4 *)(buf + node * HID) + q * 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = p[t];
}
__device__ __forceinline__ void store_acc(float *buf, size_t node, int q, const f32x4 (&v)[4]) {
  f32x4 *p = (f32x4 *)(buf + node * HID) + q * 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) p[t] = v[t];
}
__device__ __forceinline__ void add_acc(float *buf, size_t node, int q, const f32x4 (&v)[4]) {
  f32x4 *p = (f32x4 *)(buf + node * HID) + q * 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) p[t] = p[t] + v[t];
}

// BF16 node state fragments (fragment order, see gnn_common.hpp).
__device__ __forceinline__ void load_frags(const uint16_t *h, size_t node, int q, u32x4 (&f)[2]) {
  const u32x4 *p = (const u32x4 *)(h + node * HID);
  f[0] = p[q];
  f[1] = p[4 + q];
}

__device__ __forceinline__ f32x4 unpack_lo(u32x4 v) {
  return f32x4{bf16_to_f32(v.x & 0xffffu), bf16_to_f32(v.x >> 16), bf16_to_f32(v.y & 0xffffu),
               bf16_to_f32(v.y >> 16)};
}
__device__ __forceinline__ f32x4 unpack_hi(u32x4 v) {
  return f32x4{bf16_to_f32(v.z & 0xffffu), bf16_to_f32(v.z >> 16), bf16_to_f32(v.w & 0xffffu),
               bf16_to_f32(v.w >> 16)};
}

__device__ __forceinline__ uint16_t bf16_bits(float v) {
  __bf16 b = (__bf16)v;
  return __builtin_bit_cast(uint16_t, b);
}

// Staging of one value per (channel row, node column), BF16, channel-major.
// Accumulator-layout vectors: lane (n, q) holds channels 16 t + 4 q + e.
__device__ __forceinline__ void stage_acc(uint16_t *rows, const f32x4 (&v)[4], int q, int col,
                                          int row0 = 0) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    rows[(row0 + 16 * t + 4 * q + 0) * kPitch + col] = bf16_bits(v[t].x);
    rows[(row0 + 16 * t + 4 * q + 1) * kPitch + col] = bf16_bits(v[t].y);
    rows[(row0 + 16 * t + 4 * q + 2) * kPitch + col] = bf16_bits(v[t].z);
    rows[(row0 + 16 * t + 4 * q + 3) * kPitch + col] = bf16_bits(v[t].w);
  }
}
// Fragment-order vectors: element j of k-step s is channel c(s, q, j).
__device__ __forceinline__ void stage_frag(uint16_t *rows, const u32x4 (&f)[2], int q, int col,
                                           int row0 = 0) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const uint32_t w[4] = {f[s].x, f[s].y, f[s].z, f[s].w};
#pragma unroll
    for (int j = 0; j < 8; ++j)
      rows[(row0 + frag_channel(s, q, j)) * kPitch + col] =
          (uint16_t)((j & 1) ? (w[j >> 1] >> 16) : (w[j >> 1] & 0xffffu));
  }
}
__device__ __forceinline__ void stage_zero(uint16_t *rows, int nrows, int lane) {
  for (int k = lane; k < nrows * kPitch / 2; k += 64) ((uint32_t *)rows)[k] = 0u;
}

// acc[mt][ct] += D^T-slice x A over the 32 staged nodes: rows of d are the
// output channels (16 mt + ...), rows of a the input channels (16 ct + ...).
template <int MT, int CT>
__device__ __forceinline__ void dw_mma(f32x4 (&acc)[MT][CT], const uint16_t *d,
                                       const uint16_t *a, int lane) {
  const int r = lane & 15, q = lane >> 4;
  u32x4 A[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) A[mt] = *(const u32x4 *)(d + (16 * mt + r) * kPitch + 8 * q);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    u32x4 B = *(const u32x4 *)(a + (16 * ct + r) * kPitch + 8 * q);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt][ct] = mfma(A[mt], B, acc[mt][ct]);
  }
}

// Writes a dW accumulator block to this wave's partial: element
// (row 16 mt + 4 q + e, column col0 + 16 ct + (lane & 15)) of a row-major
// [rows][ld] matrix at `base`.
template <int MT, int CT>
__device__ __forceinline__ void write_dw(float *part, size_t base, int ld, int col0, int nrows,
                                         int ncols, const f32x4 (&acc)[MT][CT], int lane) {
  const int c = lane & 15, q = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const float v[4] = {acc[mt][ct].x, acc[mt][ct].y, acc[mt][ct].z, acc[mt][ct].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int row = 16 * mt + 4 * q + e, col = 16 * ct + c;
        if (row < nrows && col < ncols) part[base + (size_t)row * ld + col0 + col] = v[e];
      }
    }
}

// Sums, over the 16 node lanes, per-lane accumulator-layout vectors (channel
// 16 t + 4 q + e) and writes the 64 channel totals to part[base + stride * ch].
__device__ __forceinline__ void write_vec(float *part, size_t base, int stride,
                                          const f32x4 (&v)[4], float *red, int lane) {
  const int q = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    red[lane * 17 + 4 * t + 0] = v[t].x;
    red[lane * 17 + 4 * t + 1] = v[t].y;
    red[lane * 17 + 4 * t + 2] = v[t].z;
    red[lane * 17 + 4 * t + 3] = v[t].w;
  }
  wave_lds_sync();
  const int k = lane & 15;
  float s = 0.0f;
  for (int n = 0; n < 16; ++n) s += red[(16 * q + n) * 17 + k];
  const int ch = 16 * (k >> 2) + 4 * q + (k & 3);
  part[base + (size_t)stride * ch] = s;
  wave_lds_sync();
}

// s_waitcnt vmcnt(0) with expcnt and lgkmcnt left at their maximum.
constexpr int kBwdWaitVmcnt0 = 0x0F70;

template <int DR, int AR>
struct Stage {
  uint16_t d[DR * kPitch];
  uint16_t a[AR * kPitch];
  float red[64 * 17];
};

// ------------------------------------------------------------ the head ---

// dz from dL/dg_post at each node, dh_R = Wh^T dz, dWh, dbh.
__global__ __launch_bounds__(kBT) void bwd_head_kernel(
    const float *__restrict__ G, const float *__restrict__ gpre, const float *__restrict__ tau,
    const float *__restrict__ save_z, const uint16_t *__restrict__ hR, int batch, int nx, int ny,
    const uint8_t *__restrict__ pack, FragLayout F, BlobLayout L, float *__restrict__ dh,
    float *__restrict__ part) {
  __shared__ Stage<16, 64> st[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  Stage<16, 64> &S = st[wave];
  const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
  const float sdelta = ((const float *)(pack + F.const_off))[C_SDELTA];
  u32x4 wht[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) wht[t] = load_frag(frags, F.WHT + t, lane);
  const long long gxn = (nx + 15) / 16, ngroups = (long long)batch * ny * gxn;
  const long long nchunks = (ngroups + 1) / 2;
  const int w = blockIdx.x * 4 + wave;
  f32x4 acc[1][4] = {};
  float bsum[NOUT] = {};
  // One wave per SIMD: the next chunk's inputs (both groups) are loaded while
  // this chunk is computed; one explicit wait before the chunk's first store
  // covers them.
  float g_nx[2][9], G_nx[2][9], z_nx[2][NOUT], tau_nx[2];
  u32x4 hf_nx[2][2];
  auto prefetch = [&](long long cc) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const Pos P = group_pos(2 * cc + hh, ngroups, n, nx, ny, gxn);
      const size_t lat = (size_t)P.b * ny * 9 * nx;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        g_nx[hh][i] = gpre[lat + lbm::pidx(nx, P.y, i, P.x)];
        G_nx[hh][i] = G[lat + lbm::pidx(nx, P.y, i, P.x)];
      }
#pragma unroll
      for (int k = 0; k < NOUT; ++k) z_nx[hh][k] = save_z[P.node * 12 + k];
      tau_nx[hh] = tau[P.b];
      load_frags(hR, P.node, q, hf_nx[hh]);
    }
  };
  if (w < nchunks) prefetch(w);
  __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
  for (long long c = w; c < nchunks; c += kBwdWaves) {
    float gc[2][9], Gc[2][9], zc[2][NOUT], tauc[2];
    u32x4 hfc[2][2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        gc[hh][i] = g_nx[hh][i];
        Gc[hh][i] = G_nx[hh][i];
      }
#pragma unroll
      for (int k = 0; k < NOUT; ++k) zc[hh][k] = z_nx[hh][k];
      tauc[hh] = tau_nx[hh];
      hfc[hh][0] = hf_nx[hh][0];
      hfc[hh][1] = hf_nx[hh][1];
    }
    if (c + kBwdWaves < nchunks) prefetch(c + kBwdWaves);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      Pos P = group_pos(2 * c + half, ngroups, n, nx, ny, gxn);
      float(&g)[9] = gc[half];
      float(&Gi)[9] = Gc[half];
      float(&z)[NOUT] = zc[half];
      float drho, rho, u, v, uu;
      lbm::node_moments(g, drho, rho, u, v, uu);
      const float s = 1.0f / (1.0f + expf(-z[0]));
      const float tadj = 0.5f + s;
      const float tb = tauc[half];
      float dta = 0.0f, m0 = 0.0f, mx = 0.0f, my = 0.0f;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        dta += Gi[i] * (g[i] - lbm::geq_shifted<float>(i, drho, rho, u, v, uu));
        m0 += Gi[i];
        mx += float(cx(i)) * Gi[i];
        my += float(cy(i)) * Gi[i];
      }
      float dz[NOUT];
      dz[0] = dta / (tb * tadj * tadj) * s * (1.0f - s);
#pragma unroll
      for (int i = 0; i < 9; ++i)
        dz[1 + i] = sdelta * (Gi[i] - m0 * (1.0f / 9.0f) - float(cx(i)) * mx * (1.0f / 6.0f) -
                              float(cy(i)) * my * (1.0f / 6.0f));
      if (!P.valid)
#pragma unroll
        for (int k = 0; k < NOUT; ++k) dz[k] = 0.0f;
      // B operand: element j of lane group q is head output 8 q + j.
      float e8[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float a0 = j < NOUT ? dz[j] : 0.0f;
        float a1 = j + 8 < NOUT ? dz[(j + 8) % NOUT] : 0.0f;
        e8[j] = q == 0 ? a0 : (q == 1 ? a1 : 0.0f);
      }
      const u32x4 dzb = {pack_bf16(e8[0], e8[1]), pack_bf16(e8[2], e8[3]),
                         pack_bf16(e8[4], e8[5]), pack_bf16(e8[6], e8[7])};
      f32x4 o[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) o[t] = mfma(wht[t], dzb, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
      if (half == 0) __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
      if (P.valid) store_acc(dh, P.node, q, o);
      const u32x4 hf[2] = {hfc[half][0], hfc[half][1]};
      const int col = 16 * half + n;
#pragma unroll
      for (int k = 0; k < NOUT; ++k)
        if ((k & 3) == q) S.d[k * kPitch + col] = bf16_bits(dz[k]);
      if (q < 2)
#pragma unroll
        for (int k = NOUT; k < 16; ++k)
          if ((k & 1) == q) S.d[k * kPitch + col] = 0;
      stage_frag(S.a, hf, q, col);
      if (q == 0)
#pragma unroll
        for (int k = 0; k < NOUT; ++k) bsum[k] += dz[k];
    }
    wave_lds_sync();
    dw_mma<1, 4>(acc, S.d, S.a, lane);
    wave_lds_sync();
  }
  float *pw = part + (size_t)w * L.nparam;
  write_dw<1, 4>(pw, L.Wh, HID, 0, NOUT, HID, acc, lane);
#pragma unroll
  for (int k = 0; k < NOUT; ++k) S.red[lane * 17 + k] = q == 0 ? bsum[k] : 0.0f;
  wave_lds_sync();
  if (lane < NOUT) {
    float s = 0.0f;
    for (int m = 0; m < 16; ++m) s += S.red[m * 17 + lane];
    pw[L.bh + lane] = s;
  }
}

// ------------------------------------------------------ node update, r ---

// dp, [dh; da] = Wn^T dp, dWn, dbn.  dh_out is overwritten.
__global__ __launch_bounds__(kBT) void bwd_node_kernel(
    const float *__restrict__ dh_in, const uint16_t *__restrict__ h, const uint16_t *__restrict__ agg,
    int batch, int nx, int ny, int r, const uint8_t *__restrict__ pack, FragLayout F,
    BlobLayout L, float *__restrict__ dh_out, float *__restrict__ dagg, float *__restrict__ part) {
  __shared__ Stage<64, 128> st[4];
  __shared__ u32x4 wn_s[16 * 64], wnt_s[16 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  Stage<64, 128> &S = st[wave];
  const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
  const f32x4 *bias = (const f32x4 *)(pack + F.bias_off);
  for (int k = threadIdx.x; k < 16 * 64; k += kBT) {
    wn_s[k] = frags[(size_t)F.WN[r] * 64 + k];
    wnt_s[k] = frags[(size_t)F.WNT[r] * 64 + k];
  }
  f32x4 bn[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) bn[t] = load_bias(bias, F.BN[r] + t, lane);
  __syncthreads();
  const long long gxn = (nx + 15) / 16, ngroups = (long long)batch * ny * gxn;
  const long long nchunks = (ngroups + 1) / 2;
  const int w = blockIdx.x * 4 + wave;
  f32x4 acc[4][8] = {};
  f32x4 bsum[4] = {};
  // One wave per SIMD: each group's node state, aggregate and incoming
  // gradient are loaded while the previous group is computed, and one
  // explicit wait before the group's first store covers them (vmcnt counts
  // loads and stores together; waiting there, the loads have had most of the
  // group to land and the previous group's stores are long complete).
  u32x4 hf_nx[2], af_nx[2];
  f32x4 G_nx[4];
  auto prefetch = [&](long long grp) {
    const Pos P = group_pos(grp, ngroups, n, nx, ny, gxn);
    load_frags(h, P.node, q, hf_nx);
    load_frags(agg, P.node, q, af_nx);
    load_acc(dh_in, P.node, q, G_nx);
  };
  if (w < nchunks) prefetch(2 * (long long)w);
  __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
  for (long long c = w; c < nchunks; c += kBwdWaves) {
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
      int wo = lane;
      asm volatile("" : "+v"(wo));
      const u32x4 *wn = wn_s + wo, *wnt = wnt_s + wo;
      Pos P = group_pos(2 * c + half, ngroups, n, nx, ny, gxn);
      const u32x4 hf[2] = {hf_nx[0], hf_nx[1]}, af[2] = {af_nx[0], af_nx[1]};
      const f32x4 G[4] = {G_nx[0], G_nx[1], G_nx[2], G_nx[3]};
      if (half == 0 || c + kBwdWaves < nchunks)
        prefetch(half == 0 ? 2 * c + 1 : 2 * (c + kBwdWaves));
      f32x4 dp[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 p = mfma(wn[(4 * t) * 64], hf[0], bn[t]);
        p = mfma(wn[(4 * t + 1) * 64], hf[1], p);
        p = mfma(wn[(4 * t + 2) * 64], af[0], p);
        p = mfma(wn[(4 * t + 3) * 64], af[1], p);
        dp[t] = P.valid ? G[t] * f32x4{gelu_grad(p.x), gelu_grad(p.y), gelu_grad(p.z),
                                       gelu_grad(p.w)}
                        : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        bsum[t] += dp[t];
      }
      const u32x4 dpb[2] = {frag_from_acc(dp[0], dp[1]), frag_from_acc(dp[2], dp[3])};
      f32x4 o[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        o[t] = mfma(wnt[(2 * t) * 64], dpb[0], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        o[t] = mfma(wnt[(2 * t + 1) * 64], dpb[1], o[t]);
      }
      __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
      if (P.valid) {
        const f32x4 o_h[4] = {o[0], o[1], o[2], o[3]};
        const f32x4 o_a[4] = {o[4], o[5], o[6], o[7]};
        store_acc(dh_out, P.node, q, o_h);
        store_acc(dagg, P.node, q, o_a);
      }
      const int col = 16 * half + n;
      stage_acc(S.d, dp, q, col);
      stage_frag(S.a, hf, q, col, 0);
      stage_frag(S.a, af, q, col, HID);
    }
    wave_lds_sync();
    dw_mma<4, 8>(acc, S.d, S.a, lane);
    wave_lds_sync();
  }
  float *pw = part + (size_t)w * L.nparam;
  write_dw<4, 8>(pw, L.Wn[r], NODE_IN, 0, HID, NODE_IN, acc, lane);
  write_vec(pw, L.bn[r], 1, bsum, S.red, lane);
}

// --------------------------------------------- edge layer, receiver side ---

// Node states of one 16-receiver group and its ring (3 rows x 18 columns),
// staged in LDS: node ln = 18 hy + hx at byte 144 ln (128 B of state and 16
// B of padding, so that 16 lanes reading one 16-byte chunk of 16 consecutive
// nodes hit 16 disjoint groups of banks).  One direct-to-LDS load of a wave
// fills 64 16-byte slots, node ln's chunk c at slot 9 ln + c.
constexpr int kRingX = 18, kRingY = 3, kRingNodes = kRingX * kRingY;
constexpr int kRingNodeBytes = 144;
constexpr int kRingLoads = (kRingNodes * 9 + 63) / 64;
constexpr int kRingBytes = kRingLoads * 64 * 16;
// slot / 9 and node / 18 by multiply and shift, exact over the whole range
constexpr int kRingDiv9 = 7282, kRingDiv18 = 3641;
constexpr bool ring_divisions_exact() {
  for (int v = 0; v < kRingLoads * 64; ++v)
    if (((v * kRingDiv9) >> 16) != v / 9) return false;
  for (int v = 0; v < kRingNodes; ++v)
    if (((v * kRingDiv18) >> 16) != v / kRingX) return false;
  return true;
}
static_assert(kRingNodeBytes == 9 * 16 && ring_divisions_exact(), "ring staging");

// dq_{n,d} (stored BF16), T_n, dWa, dbe, dWc; Wa^T T_n over dL/dagg_n.
// One wave per SIMD (the kernel needs 400+ registers), so memory latency is
// hidden by prefetching instead of by other waves: while a wave works on one
// group of 16 receivers, direct-to-LDS loads bring the next group's node
// states and ring into the wave's other LDS buffer, and the next group's
// dL/dagg rows come into registers.  One explicit wait late in each
// group (vmcnt counts loads and stores together, so it also drains the
// group's earlier stores, long complete by then) covers all of them.  The
// arithmetic and its order are those of the direct loads.
__global__ __launch_bounds__(kBT) void bwd_edge_recv_kernel(
    float *__restrict__ dagg_io, const uint16_t *__restrict__ h, int batch, int nx, int ny,
    int r, const uint8_t *__restrict__ pack, FragLayout F, BlobLayout L,
    uint16_t *__restrict__ dq_out, float *__restrict__ part) {
  const float *dagg = dagg_io;
  __shared__ Stage<64, 64> st[4];
  __shared__ u32x4 wa_s[8 * 64], wat_s[8 * 64];
  __shared__ __attribute__((aligned(16))) uint8_t ring_s[4][2][kRingBytes];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  Stage<64, 64> &S = st[wave];
  const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
  const f32x4 *bias = (const f32x4 *)(pack + F.bias_off);
  for (int k = threadIdx.x; k < 8 * 64; k += kBT) {
    wa_s[k] = frags[(size_t)F.WA[r] * 64 + k];
    wat_s[k] = frags[(size_t)F.WAT[r] * 64 + k];
  }
  u32x4 wb[4][2];
  uint32_t wc[4];
  f32x4 be[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    wb[t][0] = load_frag(frags, F.WB[r] + 2 * t, lane);
    wb[t][1] = load_frag(frags, F.WB[r] + 2 * t + 1, lane);
    wc[t] = load_frag(frags, F.WC[r] + t, lane).x;
    be[t] = load_bias(bias, F.BE[r] + t, lane);
  }
  __syncthreads();
  const long long gxn = (nx + 15) / 16, ngroups = (long long)batch * ny * gxn;
  const long long nchunks = (ngroups + 1) / 2;
  const int w = blockIdx.x * 4 + wave;

  // Issues the loads of group `grp` (clamped as group_pos clamps it): its
  // ring into `buf` (direct to LDS, wrapped at the lattice edges; slots past
  // the last node repeat its last chunk) and its dL/dagg rows into registers.
  auto prefetch = [&](long long grp, uint8_t *buf, f32x4(&da)[4]) {
    const Pos P = group_pos(grp, ngroups, n, nx, ny, gxn);
    const int x0 = (int)((grp < ngroups ? grp : 0) % gxn) * 16;
    const size_t lat_nodes = (size_t)P.b * ny * nx;
#pragma unroll
    for (int k = 0; k < kRingLoads; ++k) {
      const unsigned slot = 64 * k + lane;
      unsigned ln = __umul24(slot, kRingDiv9) >> 16;
      unsigned c = slot - 9 * ln;
      if (ln >= (unsigned)kRingNodes) {
        ln = kRingNodes - 1;
        c = 7;
      }
      c = c < 7 ? c : 7;
      const int hy = (int)(__umul24(ln, kRingDiv18) >> 16);
      const int hx = (int)ln - kRingX * hy;
      int gx = x0 - 1 + hx, gy = P.y - 1 + hy;
      gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
      gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
      if (gx >= nx) gx %= nx;  // lattices narrower than the ring
      if (gy >= ny) gy %= ny;
      const uint16_t *src = h + (lat_nodes + (size_t)gy * nx + gx) * HID + c * 8;
      __builtin_amdgcn_global_load_lds((const void *)src,
                                       (__attribute__((address_space(3))) void *)(buf + k * 1024),
                                       16, 0, 0);
    }
    load_acc(dagg, P.node, q, da);
  };

  f32x4 acc[4][4] = {};
  f32x4 tsum[4] = {}, vxs[4] = {}, vys[4] = {};
  f32x4 da_nx[4];
  // One group: half 0 or 1 of chunk c, its ring in `cur`; the next group's
  // loads go to `nxt`.
  auto group = [&](long long c, int half, const uint8_t *cur, uint8_t *nxt) {
      int wo = lane;
      asm volatile("" : "+v"(wo));
      const u32x4 *wa = wa_s + wo, *wat = wat_s + wo;
      const Pos P = group_pos(2 * c + half, ngroups, n, nx, ny, gxn);
      // (zero on lanes outside the lattice)
      f32x4 da[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) da[t] = P.valid ? da_nx[t] : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      // the next group of this wave: the chunk's second half, or the first
      // half of the wave's next chunk
      // chunk q of this receiver's lower-left neighbour; every neighbour's
      // chunk is at a constant offset from it
      const uint8_t *nb = cur + n * kRingNodeBytes + q * 16;
      auto frag_at = [&](int dx, int dy, int sidx) {
        return *(const u32x4 *)(nb + ((dy + 1) * kRingX + dx + 1) * kRingNodeBytes + sidx * 64);
      };
      // all of the group's ring reads, before the next group's loads
      const u32x4 hn[2] = {frag_at(0, 0, 0), frag_at(0, 0, 1)};
      u32x4 hj[8][2];
#pragma unroll
      for (int d = 1; d < 9; ++d) {
        hj[d - 1][0] = frag_at(cx(d), cy(d), 0);
        hj[d - 1][1] = frag_at(cx(d), cy(d), 1);
      }
      f32x4 an[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        an[t] = mfma(wa[(2 * t) * 64], hn[0], be[t]);
        an[t] = mfma(wa[(2 * t + 1) * 64], hn[1], an[t]);
      }
      const long long next = half == 0 ? 2 * c + 1 : 2 * (c + kBwdWaves);
      if (half == 0 || c + kBwdWaves < nchunks) prefetch(next, nxt, da_nx);
      f32x4 T[4] = {};
      // The edge loop is unrolled in full, so the direction of each edge (its
      // edge feature, the sign it adds to the Wc gradients with) is a
      // compile-time constant and the loop has no branches to split its
      // schedule.
      const uint32_t q0 = q == 0 ? 0xffffffffu : 0u;
      // pre-activation of the message from direction d (MFMA only)
      auto message = [&](int d, f32x4(&a)[4]) {
        const u32x4 ed = {q0 & (bf16_unit(cx(d)) | (bf16_unit(cy(d)) << 16)), 0u, 0u, 0u};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a[t] = mfma(u32x4{wc[t], 0u, 0u, 0u}, ed, an[t]);
          a[t] = mfma(wb[t][0], hj[d - 1][0], a[t]);
          a[t] = mfma(wb[t][1], hj[d - 1][1], a[t]);
        }
      };
      // Software pipeline as in the forward round: the MFMA chains of edge
      // d + 1 are issued among the VALU work of edge d (one wave per SIMD
      // here, so nothing else fills the matrix-core latency).  The sums run
      // over d in the same order as without the pipeline.
      f32x4 pre[2][4];
      message(1, pre[1]);
#pragma unroll
      for (int d = 1; d < 9; ++d) {
        if (d < 8) message(d + 1, pre[(d + 1) & 1]);
        f32x4 dq[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const f32x4 a = pre[d & 1][t];
          dq[t] = da[t] * f32x4{gelu_grad(a.x), gelu_grad(a.y), gelu_grad(a.z), gelu_grad(a.w)};
          T[t] += dq[t];
          if (cx(d) > 0) vxs[t] += dq[t];
          if (cx(d) < 0) vxs[t] -= dq[t];
          if (cy(d) > 0) vys[t] += dq[t];
          if (cy(d) < 0) vys[t] -= dq[t];
        }
        // The next group's loads were issued at the start of this one: wait
        // for them here, where they have had most of the group to land.
        // Unconditional, so the compiler also counts them as complete.
        if (d == 6) __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
        if (P.valid) {
          // non-temporal: 1 KB per node, read back once by the sender side
          // (measured: the sender side then runs 18 % faster, this kernel 4 %
          // slower)
          u32x4 *o = (u32x4 *)(dq_out + (P.node * 8 + (d - 1)) * HID);
          __builtin_nontemporal_store(frag_from_acc(dq[0], dq[1]), o + q);
          __builtin_nontemporal_store(frag_from_acc(dq[2], dq[3]), o + 4 + q);
        }
        if (d < 8) {
          // each of edge d + 1's 12 MFMAs followed by 10 VALU instructions
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);
          }
        }
      }
      const u32x4 tb[2] = {frag_from_acc(T[0], T[1]), frag_from_acc(T[2], T[3])};
      f32x4 o[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        o[t] = mfma(wat[(2 * t) * 64], tb[0], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        o[t] = mfma(wat[(2 * t + 1) * 64], tb[1], o[t]);
        tsum[t] += T[t];
      }
      // Wa^T T replaces this group's dL/dagg rows, read by nobody after
      // this group; the sender-side kernel adds it to dh.
      if (P.valid) store_acc(dagg_io, P.node, q, o);
      const int col = 16 * half + n;
      stage_acc(S.d, T, q, col);
      stage_frag(S.a, hn, q, col);
  };

  // Group i of this wave works from ring_s[wave][i % 2].  The compiler
  // cannot tell the two buffers apart, so it would wait for loads in flight
  // into one before any LDS read: each group therefore does all its ring and
  // Wa reads before it issues the next group's loads, and reads LDS again
  // only after its explicit wait.
  if (w < nchunks) prefetch(2 * (long long)w, ring_s[wave][0], da_nx);
  __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
  for (long long c = w; c < nchunks; c += kBwdWaves) {
#pragma unroll 1
    for (int half = 0; half < 2; ++half) group(c, half, ring_s[wave][half], ring_s[wave][half ^ 1]);
    wave_lds_sync();
    dw_mma<4, 4>(acc, S.d, S.a, lane);
    wave_lds_sync();
  }
  float *pw = part + (size_t)w * L.nparam;
  write_dw<4, 4>(pw, L.We[r], EDGE_IN, 0, HID, HID, acc, lane);
  write_vec(pw, L.be[r], 1, tsum, S.red, lane);
  write_vec(pw, L.We[r] + 2 * HID, EDGE_IN, vxs, S.red, lane);
  write_vec(pw, L.We[r] + 2 * HID + 1, EDGE_IN, vys, S.red, lane);
}

// ----------------------------------------------- edge layer, sender side ---

// S_m = sum_d dq_{m - e_d, d}; dWb; dh_m += Wa^T T_m (left by the receiver
// side in orecv), then dh_m += Wb^T S_m.
__global__ __launch_bounds__(kBT) void bwd_edge_send_kernel(
    const uint16_t *__restrict__ dq_in, const uint16_t *__restrict__ h, int batch, int nx,
    int ny, int r, const uint8_t *__restrict__ pack, FragLayout F, BlobLayout L,
    const float *__restrict__ orecv, float *__restrict__ dh, float *__restrict__ part) {
  __shared__ Stage<64, 64> st[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  Stage<64, 64> &S = st[wave];
  const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
  u32x4 wbt[4][2];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    wbt[t][0] = load_frag(frags, F.WBT[r] + 2 * t, lane);
    wbt[t][1] = load_frag(frags, F.WBT[r] + 2 * t + 1, lane);
  }
  const long long gxn = (nx + 15) / 16, ngroups = (long long)batch * ny * gxn;
  const long long nchunks = (ngroups + 1) / 2;
  const int w = blockIdx.x * 4 + wave;
  f32x4 acc[4][4] = {};
  // One wave per SIMD: the next group's dq rows (eight directions), node
  // state, dh and the receiver side's term are loaded while this group is
  // computed; one explicit wait before the group's store covers them.
  u32x4 dq_nx[8][2], hm_nx[2];
  f32x4 dh_nx[4], or_nx[4];
  auto prefetch = [&](long long grp) {
    const Pos P = group_pos(grp, ngroups, n, nx, ny, gxn);
    const size_t lat_nodes = (size_t)P.b * ny * nx;
#pragma unroll
    for (int d = 1; d < 9; ++d) {
      int xn = P.x - cx(d), yn = P.y - cy(d);  // receiver whose edge d points here
      xn = xn < 0 ? xn + nx : (xn >= nx ? xn - nx : xn);
      yn = yn < 0 ? yn + ny : (yn >= ny ? yn - ny : yn);
      const u32x4 *src =
          (const u32x4 *)(dq_in + ((lat_nodes + (size_t)yn * nx + xn) * 8 + (d - 1)) * HID);
      dq_nx[d - 1][0] = __builtin_nontemporal_load(src + q);  // read once
      dq_nx[d - 1][1] = __builtin_nontemporal_load(src + 4 + q);
    }
    load_frags(h, P.node, q, hm_nx);
    load_acc(dh, P.node, q, dh_nx);
    load_acc(orecv, P.node, q, or_nx);
  };
  if (w < nchunks) prefetch(2 * (long long)w);
  __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
  for (long long c = w; c < nchunks; c += kBwdWaves) {
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
      Pos P = group_pos(2 * c + half, ngroups, n, nx, ny, gxn);
      u32x4 dqc[8][2], hm[2];
      f32x4 dhc[4], orc[4];
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        dqc[d][0] = dq_nx[d][0];
        dqc[d][1] = dq_nx[d][1];
      }
      hm[0] = hm_nx[0];
      hm[1] = hm_nx[1];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        dhc[t] = dh_nx[t];
        orc[t] = or_nx[t];
      }
      if (half == 0 || c + kBwdWaves < nchunks)
        prefetch(half == 0 ? 2 * c + 1 : 2 * (c + kBwdWaves));
      f32x4 Sm[4] = {};
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        Sm[0] += unpack_lo(dqc[d][0]);
        Sm[1] += unpack_hi(dqc[d][0]);
        Sm[2] += unpack_lo(dqc[d][1]);
        Sm[3] += unpack_hi(dqc[d][1]);
      }
      if (!P.valid)
#pragma unroll
        for (int t = 0; t < 4; ++t) Sm[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      const u32x4 sb[2] = {frag_from_acc(Sm[0], Sm[1]), frag_from_acc(Sm[2], Sm[3])};
      f32x4 o[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        o[t] = mfma(wbt[t][0], sb[0], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        o[t] = mfma(wbt[t][1], sb[1], o[t]);
      }
      __builtin_amdgcn_s_waitcnt(kBwdWaitVmcnt0);
      if (P.valid) {
        f32x4 *p = (f32x4 *)(dh + P.node * HID) + q * 4;
#pragma unroll
        for (int t = 0; t < 4; ++t) p[t] = (dhc[t] + orc[t]) + o[t];
      }
      const int col = 16 * half + n;
      stage_acc(S.d, Sm, q, col);
      stage_frag(S.a, hm, q, col);
    }
    wave_lds_sync();
    dw_mma<4, 4>(acc, S.d, S.a, lane);
    wave_lds_sync();
  }
  float *pw = part + (size_t)w * L.nparam;
  write_dw<4, 4>(pw, L.We[r], EDGE_IN, HID, HID, HID, acc, lane);
}

// ------------------------------------------------------------- encoder ---

// Derivative of the activation at the recomputed pre-activation: GELU (tanh
// form) for the message-passing network, ReLU (1 for p > 0, else 0) for the
// per-node network of Fig. 2.
template <int ACT>
__device__ __forceinline__ f32x4 act_grad4(f32x4 p) {
  if constexpr (ACT == 0)
    return f32x4{gelu_grad(p.x), gelu_grad(p.y), gelu_grad(p.z), gelu_grad(p.w)};
  else
    return f32x4{p.x > 0.0f ? 1.0f : 0.0f, p.y > 0.0f ? 1.0f : 0.0f, p.z > 0.0f ? 1.0f : 0.0f,
                 p.w > 0.0f ? 1.0f : 0.0f};
}

template <int ACT>
__global__ __launch_bounds__(kBT) void bwd_encoder_kernel(
    const float *__restrict__ dh0, const uint16_t *__restrict__ sx, const uint16_t *__restrict__ se1,
    int batch, int nx, int ny, const uint8_t *__restrict__ pack, FragLayout F, BlobLayout L,
    float *__restrict__ part) {
  __shared__ Stage<64, 64> st[4];
  __shared__ uint16_t d1s[4][64 * kPitch], x1s[4][16 * kPitch];
  __shared__ u32x4 w2t_s[8 * 64], w1_s[4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, q = lane >> 4;
  Stage<64, 64> &S = st[wave];
  uint16_t *D1 = d1s[wave], *X1 = x1s[wave];
  const u32x4 *frags = (const u32x4 *)(pack + F.frag_off);
  const f32x4 *bias = (const f32x4 *)(pack + F.bias_off);
  // W2^T and W1 are read from LDS inside the loop, so that the loop issues
  // no global loads besides its node data
  for (int k = threadIdx.x; k < 8 * 64; k += kBT) w2t_s[k] = frags[(size_t)F.W2T * 64 + k];
  for (int k = threadIdx.x; k < 4 * 64; k += kBT) w1_s[k] = frags[(size_t)F.W1 * 64 + k];
  u32x4 w2[4][2];
  f32x4 b1[4], b2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    w2[t][0] = load_frag(frags, F.W2 + 2 * t, lane);
    w2[t][1] = load_frag(frags, F.W2 + 2 * t + 1, lane);
    b1[t] = load_bias(bias, F.B1 + t, lane);
    b2[t] = load_bias(bias, F.B2 + t, lane);
  }
  const long long gxn = (nx + 15) / 16, ngroups = (long long)batch * ny * gxn;
  const long long nchunks = (ngroups + 1) / 2;
  const int w = blockIdx.x * 4 + wave;
  __syncthreads();
  f32x4 acc2[4][4] = {}, acc1[4][1] = {};
  f32x4 s1[4] = {}, s2[4] = {};
  // One wave per SIMD: the next group's first-layer output, features and
  // incoming gradient are loaded while this group is computed (the loop has
  // no stores, so the compiler's in-order load counts cover them).
  u32x4 e1_nx[2], xb_nx;
  f32x4 G_nx[4];
  auto prefetch = [&](long long grp) {
    const Pos P = group_pos(grp, ngroups, n, nx, ny, gxn);
    load_frags(se1, P.node, q, e1_nx);
    xb_nx = q < 2 ? ((const u32x4 *)(sx + P.node * 16))[q] : u32x4{0u, 0u, 0u, 0u};
    load_acc(dh0, P.node, q, G_nx);
  };
  if (w < nchunks) prefetch(2 * (long long)w);
  for (long long c = w; c < nchunks; c += kBwdWaves) {
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
      int wo = lane;
      asm volatile("" : "+v"(wo));
      Pos P = group_pos(2 * c + half, ngroups, n, nx, ny, gxn);
      const u32x4 e1[2] = {e1_nx[0], e1_nx[1]};
      const u32x4 xb = xb_nx;
      const f32x4 G[4] = {G_nx[0], G_nx[1], G_nx[2], G_nx[3]};
      if (half == 0 || c + kBwdWaves < nchunks)
        prefetch(half == 0 ? 2 * c + 1 : 2 * (c + kBwdWaves));
      f32x4 dp2[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 p = mfma(w2[t][0], e1[0], b2[t]);
        p = mfma(w2[t][1], e1[1], p);
        dp2[t] = P.valid ? G[t] * act_grad4<ACT>(p) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        s2[t] += dp2[t];
      }
      const u32x4 dpb[2] = {frag_from_acc(dp2[0], dp2[1]), frag_from_acc(dp2[2], dp2[3])};
      f32x4 dp1[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 de1 = mfma(w2t_s[(2 * t) * 64 + wo], dpb[0], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        de1 = mfma(w2t_s[(2 * t + 1) * 64 + wo], dpb[1], de1);
        f32x4 p1 = mfma(w1_s[t * 64 + wo], xb, b1[t]);
        dp1[t] = de1 * act_grad4<ACT>(p1);
        s1[t] += dp1[t];
      }
      const int col = 16 * half + n;
      stage_acc(S.d, dp2, q, col);
      stage_frag(S.a, e1, q, col);
      stage_acc(D1, dp1, q, col);
      // feature rows k = 8 q + j (12 used; rows 12..15 hold zero features)
      if (q < 2) {
        const uint32_t wv[4] = {xb.x, xb.y, xb.z, xb.w};
#pragma unroll
        for (int j = 0; j < 8; ++j)
          X1[(8 * q + j) * kPitch + col] =
              (uint16_t)((j & 1) ? (wv[j >> 1] >> 16) : (wv[j >> 1] & 0xffffu));
      }
    }
    wave_lds_sync();
    dw_mma<4, 4>(acc2, S.d, S.a, lane);
    dw_mma<4, 1>(acc1, D1, X1, lane);
    wave_lds_sync();
  }
  float *pw = part + (size_t)w * L.nparam;
  write_dw<4, 4>(pw, L.W2, HID, 0, HID, HID, acc2, lane);
  write_dw<4, 1>(pw, L.W1, NFEAT, 0, HID, NFEAT, acc1, lane);
  write_vec(pw, L.b2, 1, s2, S.red, lane);
  write_vec(pw, L.b1, 1, s1, S.red, lane);
}

// Fixed-order sum of the per-wave partials: one thread per parameter, the
// partials added in wave order.  One-wave blocks spread the ~600 waves over
// every CU, and the unrolled loop keeps 32 independent loads in flight ahead
// of the (sequential) additions.
constexpr int kReduceThreads = 64;
__global__ __launch_bounds__(kReduceThreads) void bwd_reduce_kernel(
    const float *__restrict__ part, size_t nparam, float *__restrict__ grad) {
  size_t p = (size_t)blockIdx.x * kReduceThreads + threadIdx.x;
  if (p >= nparam) return;
  float s = 0.0f;
#pragma unroll 32
  for (int w = 0; w < kBwdWaves; ++w) s += part[(size_t)w * nparam + p];
  grad[p] = s;
}

// ------------------------------------------------------------ MSE, Adam ---

__global__ __launch_bounds__(kBT) void mse_kernel(const float *__restrict__ a,
                                                  const float *__restrict__ b, size_t n,
                                                  float gscale, float *__restrict__ grad,
                                                  double *__restrict__ partials) {
  __shared__ double sm[kBT];
  double s = 0.0;
  for (size_t k = (size_t)blockIdx.x * kBT + threadIdx.x; k < n; k += (size_t)gridDim.x * kBT) {
    float d = a[k] - b[k];
    s += (double)d * (double)d;
    if (grad) grad[k] = gscale * d;
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int k = kBT / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}

// Eq. 4 with the residual weighted by a symmetric 9 x 9 matrix Q per node:
// sum over nodes of r^T Q r, r = a - b over the nine populations of a node
// (row-interleaved layout [batch][ny][9][nx]); gradient gscale * Q r.  The
// products with Q are taken in FP64.
struct MseWeights {
  double q[81];
};

__global__ __launch_bounds__(kBT) void mse_weighted_kernel(const float *__restrict__ a,
                                                           const float *__restrict__ b,
                                                           int batch, int nx, int ny,
                                                           MseWeights Q, float gscale,
                                                           float *__restrict__ grad,
                                                           double *__restrict__ partials) {
  __shared__ double sm[kBT];
  double s = 0.0;
  const size_t nodes = (size_t)batch * ny * nx;
  for (size_t k = (size_t)blockIdx.x * kBT + threadIdx.x; k < nodes;
       k += (size_t)gridDim.x * kBT) {
    const size_t row = k / (size_t)nx, x = k - row * nx;     // row = b * ny + y
    const size_t base = row * 9 * (size_t)nx + x;
    double r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = (double)a[base + (size_t)i * nx] - (double)b[base + (size_t)i * nx];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < 9; ++j) t += Q.q[9 * i + j] * r[j];
      s += r[i] * t;
      if (grad) grad[base + (size_t)i * nx] = gscale * (float)t;
    }
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int k = kBT / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kBT) void mse_finalize(const double *__restrict__ partials, int nb,
                                                    double scale, double *__restrict__ loss) {
  __shared__ double sm[kBT];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += kBT) s += partials[k];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int k = kBT / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = scale * sm[0];
}

__global__ __launch_bounds__(kBT) void adam_kernel(float *__restrict__ p,
                                                   const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   size_t n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
  size_t k = (size_t)blockIdx.x * kBT + threadIdx.x;
  if (k >= n) return;
  float gk = g[k];
  float mk = b1 * m[k] + (1.0f - b1) * gk;
  float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace gnn

// ------------------------------------------------------------------- ABI ---

using namespace gnn;
using lbm::check_device;
using lbm::fail;
using lbm::launch_check;

static inline void *at(void *base, size_t off) { return (uint8_t *)base + off; }
static inline const void *at(const void *base, size_t off) {
  return (const uint8_t *)base + off;
}

extern "C" int gnn_backward(const float *dL_dgpost, const float *g_pre, const void *saved,
                            int batch, int nx, int ny, const float *tau, const float *params,
                            int n_rounds, float *grad, void *workspace, size_t ws_bytes,
                            void *stream) {
  const int R = n_rounds;
  if (!dL_dgpost || !g_pre || !saved || !tau || !params || !grad)
    return fail(LBM_EINVAL, "gnn_backward: null pointer");
  if (R < 0 || R > MAX_ROUNDS) return fail(LBM_EINVAL, "gnn_backward: bad n_rounds %d", R);
  if (batch < 1 || !lbm::lattice_ok(nx, ny) || (long long)batch * nx * ny >= (1LL << 31))
    return fail(LBM_EINVAL, "gnn_backward: bad sizes");
  const long long nodes = (long long)batch * nx * ny;
  const size_t need = backward_workspace_bytes(batch, nx, ny, R);
  if (!workspace || ws_bytes < need)
    return fail(LBM_EWORKSPACE, "gnn_backward: workspace needs %zu bytes", need);
  if (int rc = check_device()) return rc;
  hipStream_t s = (hipStream_t)stream;
  const BlobLayout L = blob_layout(R);
  const FragLayout F = frag_layout(R);
  const BackwardScratch W = backward_scratch(nodes, R);
  const SavedLayout SL = saved_layout(nodes, R);
  uint8_t *pack = (uint8_t *)at(workspace, W.pack);
  if (int rc = launch_prep(params, R, pack, nullptr, s)) return rc;
  float *part = (float *)at(workspace, W.part);
  float *dh[2] = {(float *)at(workspace, W.dhA), (float *)at(workspace, W.dhB)};
  float *dagg = (float *)at(workspace, W.dagg);
  uint16_t *dq = (uint16_t *)at(workspace, W.dq);
  const size_t hstride = align256((size_t)nodes * HID * 2);
  auto hsaved = [&](int r) { return (const uint16_t *)at(saved, SL.h + (size_t)r * hstride); };
  auto asaved = [&](int r) { return (const uint16_t *)at(saved, SL.agg + (size_t)r * hstride); };

  int cur = 0;
  hipLaunchKernelGGL(bwd_head_kernel, dim3(kBwdBlocks), dim3(kBT), 0, s, dL_dgpost, g_pre, tau,
                     (const float *)at(saved, SL.z), hsaved(R), batch, nx, ny, pack, F, L,
                     dh[cur], part);
  if (int rc = launch_check("bwd_head_kernel")) return rc;
  for (int r = R - 1; r >= 0; --r) {
    float *din = dh[cur], *dout = dh[cur ^ 1];
    hipLaunchKernelGGL(bwd_node_kernel, dim3(kBwdBlocks), dim3(kBT), 0, s, din, hsaved(r),
                       asaved(r), batch, nx, ny, r, pack, F, L, dout, dagg, part);
    if (int rc = launch_check("bwd_node_kernel")) return rc;
    hipLaunchKernelGGL(bwd_edge_recv_kernel, dim3(kBwdBlocks), dim3(kBT), 0, s, dagg, hsaved(r),
                       batch, nx, ny, r, pack, F, L, dq, part);
    if (int rc = launch_check("bwd_edge_recv_kernel")) return rc;
    hipLaunchKernelGGL(bwd_edge_send_kernel, dim3(kBwdBlocks), dim3(kBT), 0, s, dq, hsaved(r),
                       batch, nx, ny, r, pack, F, L, dagg, dout, part);
    if (int rc = launch_check("bwd_edge_send_kernel")) return rc;
    cur ^= 1;
  }
  // n_rounds = 0 is the per-node network of Fig. 2, which uses ReLU
  if (R == 0)
    hipLaunchKernelGGL(bwd_encoder_kernel<1>, dim3(kBwdBlocks), dim3(kBT), 0, s, dh[cur],
                       (const uint16_t *)at(saved, SL.x), (const uint16_t *)at(saved, SL.e1),
                       batch, nx, ny, pack, F, L, part);
  else
    hipLaunchKernelGGL(bwd_encoder_kernel<0>, dim3(kBwdBlocks), dim3(kBT), 0, s, dh[cur],
                       (const uint16_t *)at(saved, SL.x), (const uint16_t *)at(saved, SL.e1),
                       batch, nx, ny, pack, F, L, part);
  if (int rc = launch_check("bwd_encoder_kernel")) return rc;
  hipLaunchKernelGGL(bwd_reduce_kernel,
                     dim3((unsigned)((L.nparam + kReduceThreads - 1) / kReduceThreads)),
                     dim3(kReduceThreads), 0, s, part, L.nparam, grad);
  return launch_check("bwd_reduce_kernel");
}

extern "C" int gnn_mse(const float *a, const float *b, int batch, int nx, int ny, double scale,
                       double *loss, float *grad_a, void *workspace, size_t ws_bytes,
                       void *stream) {
  if (!a || !b || !loss) return fail(LBM_EINVAL, "gnn_mse: null pointer");
  if (batch < 1 || !lbm::lattice_ok(nx, ny)) return fail(LBM_EINVAL, "gnn_mse: bad sizes");
  const long long nodes = (long long)batch * nx * ny;
  const int nb = lbm::reduce_blocks(nodes);
  if (!workspace || ws_bytes < (size_t)nb * 8 * sizeof(double))
    return fail(LBM_EWORKSPACE, "gnn_mse: workspace needs %zu bytes",
                (size_t)nb * 8 * sizeof(double));
  if (int rc = check_device()) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)nodes * 9;
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(kBT), 0, s, a, b, n,
                     (float)(2.0 * scale / (double)nodes), grad_a, (double *)workspace);
  if (int rc = launch_check("mse_kernel")) return rc;
  hipLaunchKernelGGL(mse_finalize, dim3(1), dim3(kBT), 0, s, (const double *)workspace, nb,
                     scale / (double)nodes, loss);
  return launch_check("mse_finalize");
}

extern "C" int gnn_mse_weighted(const float *a, const float *b, int batch, int nx, int ny,
                                const double *q, double scale, double *loss, float *grad_a,
                                void *workspace, size_t ws_bytes, void *stream) {
  if (!a || !b || !loss || !q) return fail(LBM_EINVAL, "gnn_mse_weighted: null pointer");
  if (batch < 1 || !lbm::lattice_ok(nx, ny) || (long long)batch * nx * ny >= (1LL << 31))
    return fail(LBM_EINVAL, "gnn_mse_weighted: bad sizes");
  MseWeights Q;
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      const double v = q[9 * i + j];
      if (!(fabs(v) < INFINITY) || v != q[9 * j + i])
        return fail(LBM_EINVAL, "gnn_mse_weighted: Q must be finite and symmetric");
      Q.q[9 * i + j] = v;
    }
  const long long nodes = (long long)batch * nx * ny;
  const int nb = lbm::reduce_blocks(nodes);
  if (!workspace || ws_bytes < (size_t)nb * 8 * sizeof(double))
    return fail(LBM_EWORKSPACE, "gnn_mse_weighted: workspace needs %zu bytes",
                (size_t)nb * 8 * sizeof(double));
  if (int rc = check_device()) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(mse_weighted_kernel, dim3(nb), dim3(kBT), 0, s, a, b, batch, nx, ny, Q,
                     (float)(2.0 * scale / (double)nodes), grad_a, (double *)workspace);
  if (int rc = launch_check("mse_weighted_kernel")) return rc;
  hipLaunchKernelGGL(mse_finalize, dim3(1), dim3(kBT), 0, s, (const double *)workspace, nb,
                     scale / (double)nodes, loss);
  return launch_check("mse_finalize");
}

extern "C" int gnn_adam(float *params, const float *grad, float *m, float *v, size_t n, float lr,
                        float beta1, float beta2, float eps, int step, void *stream) {
  if (!params || !grad || !m || !v) return fail(LBM_EINVAL, "gnn_adam: null pointer");
  if (step < 1) return fail(LBM_EINVAL, "gnn_adam: step must be >= 1");
  if (n == 0) return LBM_OK;
  if (int rc = check_device()) return rc;
  const double c1 = 1.0 - pow((double)beta1, step), c2 = 1.0 - pow((double)beta2, step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + kBT - 1) / kBT)), dim3(kBT), 0,
                     (hipStream_t)stream, params, grad, m, v, n, lr, beta1, beta2, eps,
                     (float)c1, (float)c2);
  return launch_check("adam_kernel");
}
