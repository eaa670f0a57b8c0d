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
// Weight fragments and the collision epilogue are shared with the
// message-passing kernels (gnn_common.hpp, gnn_collide).
#include "gnn_common.hpp"
#include "lbm_common.hpp"

namespace gnn {

// Shared with gnn_kernels.hip.
int launch_prep(const float *params, int R, uint8_t *pack, hipStream_t s);

namespace simple {

using lbm::cx;
using lbm::cy;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <bool PULL>
__device__ __forceinline__ void pops(const float *__restrict__ lat, int nx, int ny, int x, int y,
                                     float (&g)[9]) {
  if constexpr (PULL) {
    lbm::pull9(lat, nx, ny, x, y, g);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = lat[lbm::pidx(nx, y, i, x)];
  }
}

__device__ __forceinline__ f32x4 relu4(f32x4 v) {
  return f32x4{v.x > 0.0f ? v.x : 0.0f, v.y > 0.0f ? v.y : 0.0f, v.z > 0.0f ? v.z : 0.0f,
               v.w > 0.0f ? v.w : 0.0f};
}

// Eq. 3 with the projected correction at one node (same arithmetic as the
// message-passing head).
__device__ __forceinline__ void collide(float (&g)[9], const float (&z)[NOUT], float tau,
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
  for (int i = 0; i < 9; ++i) {
    float relaxed = g[i] + omega * (lbm::geq_shifted<float>(i, drho, rho, u, v, uu) - g[i]);
    float df = z[1 + i] - m0 - float(cx(i)) * mx - float(cy(i)) * my;
    g[i] = relaxed + sdelta * df;
  }
}

// A wave takes 64 consecutive nodes of one lattice row, grid-stride, one
// node per lane for everything that is per node: the coalesced pull of the
// nine populations (kept in registers for the collision), the moments and the
// 12 normalised features (rounded to BF16 into a wave-private LDS slot), and
// the collision.  The network runs in between on MFMA, four column blocks of
// 16 nodes with lane (n, q) = (node, channel group); the head outputs go back
// to one node per lane through LDS.  Weights sit in LDS so that the kernel
// keeps enough waves in flight to hide the loads.
constexpr int kZStride = NOUT + 1;   // odd stride: the 64 lanes' z rows spread over banks

template <bool PULL>
__global__ __launch_bounds__(kThreads) void simple_step_kernel(
    const float *__restrict__ src, float *__restrict__ dst, int batch, int nx, int ny,
    const float *__restrict__ tau_arr, float tau_s, const uint8_t *__restrict__ pack,
    FragLayout F, float *__restrict__ head_out, double *__restrict__ pmass,
    unsigned *__restrict__ pflag) {
  __shared__ u32x4 w_s[14 * 64];               // W1 (4), W2 (8), Wh (2) fragments
  __shared__ f32x4 b_s[9 * 64];                // b1 (4), b2 (4), bh (1)
  __shared__ uint32_t feat_s[kWaves][64 * 8];  // 16 BF16 features per node (12 used)
  __shared__ float zb[kWaves][64 * kZStride];
  __shared__ double red_m[kThreads];
  __shared__ unsigned red_f[kThreads];
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
    for (int k = threadIdx.x; k < 9 * 64; k += kThreads) {
      int b = k >> 6, l = k & 63;
      int src_b = b < 4 ? F.B1 + b : (b < 8 ? F.B2 + (b - 4) : F.BH);
      b_s[k] = bias[(size_t)src_b * 64 + l];
    }
  }
  const float *cst = (const float *)(pack + F.const_off);
  const float sdelta = cst[C_SDELTA];
  float mu[NFEAT], isg[NFEAT];
#pragma unroll
  for (int k = 0; k < NFEAT; ++k) {
    mu[k] = cst[C_MU + k];
    isg[k] = 1.0f / cst[C_SIGMA + k];
  }
  __syncthreads();
  uint32_t *fw = feat_s[wave];
  float *z_w = zb[wave];
  double mass_acc = 0.0;
  unsigned flag_acc = 0;

  const long long cxn = (nx + 63) / 64;
  const long long nchunks = (long long)batch * ny * cxn;
  for (long long c = (long long)blockIdx.x * kWaves + wave; c < nchunks;
       c += (long long)gridDim.x * kWaves) {
    const int xc = (int)(c % cxn);
    const long long by = c / cxn;
    const int y = (int)(by % ny), b = (int)(by / ny);
    const size_t lat_off = (size_t)b * ny * 9 * nx;
    const float *lat = src + lat_off;
    const int x = xc * 64 + lane;
    const bool valid = x < nx;
    float gp[9];
    pops<PULL>(lat, nx, ny, valid ? x : x % nx, y, gp);
    {
      float drho, rho, u, v, uu;
      lbm::node_moments(gp, drho, rho, u, v, uu);
      const float raw[NFEAT] = {gp[0], gp[1], gp[2], gp[3], gp[4], gp[5],
                                gp[6], gp[7], gp[8], drho, u,     v};
      float ft[NFEAT];
#pragma unroll
      for (int k = 0; k < NFEAT; ++k) ft[k] = (raw[k] - mu[k]) * isg[k];
      u32x4 *o = (u32x4 *)(fw + lane * 8);
      o[0] = u32x4{pack_bf16(ft[0], ft[1]), pack_bf16(ft[2], ft[3]), pack_bf16(ft[4], ft[5]),
                   pack_bf16(ft[6], ft[7])};
      o[1] = u32x4{pack_bf16(ft[8], ft[9]), pack_bf16(ft[10], ft[11]), 0u, 0u};
    }
    wave_lds_sync();
#pragma unroll 1
    for (int grp = 0; grp < 4; ++grp) {
      int wo = lane;
      asm volatile("" : "+v"(wo));
      const u32x4 *w = w_s + wo;
      const f32x4 *bs = b_s + wo;
      const u32x4 xb = q < 2 ? *(const u32x4 *)(fw + (16 * grp + n) * 8 + 4 * q)
                             : u32x4{0u, 0u, 0u, 0u};
      f32x4 a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = relu4(mfma(w[t * 64], xb, bs[t * 64]));
      const u32x4 e1[2] = {frag_from_acc(a[0], a[1]), frag_from_acc(a[2], a[3])};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        a[t] = relu4(mfma(w[(5 + 2 * t) * 64], e1[1],
                          mfma(w[(4 + 2 * t) * 64], e1[0], bs[(4 + t) * 64])));
      const u32x4 hb[2] = {frag_from_acc(a[0], a[1]), frag_from_acc(a[2], a[3])};
      const f32x4 z = mfma(w[13 * 64], hb[1], mfma(w[12 * 64], hb[0], bs[8 * 64]));
      const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int k = 4 * q + e;
        if (k < NOUT) z_w[(16 * grp + n) * kZStride + k] = zz[e];
      }
    }
    wave_lds_sync();
    if (valid) {
      float z[NOUT];
#pragma unroll
      for (int k = 0; k < NOUT; ++k) z[k] = z_w[lane * kZStride + k];
      const float tau = tau_arr ? tau_arr[b] : tau_s;
      collide(gp, z, tau, sdelta);
      float *d = dst + lat_off + (size_t)y * 9 * nx + x;
      double msum = 0.0;
      unsigned bad = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        __builtin_nontemporal_store(gp[i], d + (size_t)i * nx);
        float f = gp[i] + lbm::wgt<float>(i);
        bad |= (f >= 0.0f && f < INFINITY) ? 0u : 1u;
        msum += (double)gp[i];
      }
      mass_acc += msum;
      flag_acc |= bad;
      if (head_out) {
        const size_t node = ((size_t)b * ny + y) * nx + x;
        for (int k = 0; k < NOUT; ++k) head_out[node * NOUT + k] = z[k];
      }
    }
    wave_lds_sync();
  }

  red_m[threadIdx.x] = mass_acc;
  red_f[threadIdx.x] = flag_acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red_m[threadIdx.x] += red_m[threadIdx.x + s];
      red_f[threadIdx.x] |= red_f[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pmass[blockIdx.x] = red_m[0];
    pflag[blockIdx.x] = red_f[0];
  }
}

}  // namespace simple

// Gate kernels of the message-passing step (gnn_kernels.hip).
int launch_gate(const float *g_src, float *g_dst, int nx, int ny, float tau,
                const lbm_fallback *fb, int nparts, void *pmass, void *pflag, void *pmass2,
                void *ctrl, hipStream_t s);

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

static int launch_simple(bool pull, const float *src, float *dst, int batch, int nx, int ny,
                         const float *tau_arr, float tau, const float *params, float *head_out,
                         void *ws, hipStream_t s, int &nparts) {
  const FragLayout F = frag_layout(0);
  const SimpleScratch W = simple_scratch();
  uint8_t *pack = (uint8_t *)at_(ws, W.pack);
  if (int rc = launch_prep(params, 0, pack, s)) return rc;
  const long long chunks = (long long)batch * ny * ((nx + 63) / 64);
  long long blocks = (chunks + simple::kWaves - 1) / simple::kWaves;
  long long cap = (long long)simple_device_cus() * 8;
  if (cap > kMaxGnnBlocks) cap = kMaxGnnBlocks;
  const int nb = (int)(blocks < cap ? blocks : cap);
  nparts = nb;
  double *pm = (double *)at_(ws, W.pmass);
  unsigned *pf = (unsigned *)at_(ws, W.pflag);
  if (pull)
    hipLaunchKernelGGL(simple::simple_step_kernel<true>, dim3(nb), dim3(simple::kThreads), 0, s,
                       src, dst, batch, nx, ny, tau_arr, tau, pack, F, head_out, pm, pf);
  else
    hipLaunchKernelGGL(simple::simple_step_kernel<false>, dim3(nb), dim3(simple::kThreads), 0,
                       s, src, dst, batch, nx, ny, tau_arr, tau, pack, F, head_out, pm, pf);
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
                              void *workspace, size_t ws_bytes, void *stream) {
  if (int rc = check_simple("simple_forward", batch, nx, ny, params)) return rc;
  if (!g_pre || !g_post || !tau) return fail(LBM_EINVAL, "simple_forward: null pointer");
  if (lbm::overlap(g_pre, g_post, (size_t)batch * 9 * nx * ny * sizeof(float)))
    return fail(LBM_EINVAL, "simple_forward: g_pre and g_post overlap");
  if (!workspace || ws_bytes < simple_scratch().total)
    return fail(LBM_EWORKSPACE, "simple_forward: workspace needs %zu bytes",
                simple_scratch().total);
  if (int rc = check_device()) return rc;
  int nparts = 0;
  return launch_simple(false, g_pre, g_post, batch, nx, ny, tau, 0.0f, params, head_out,
                       workspace, (hipStream_t)stream, nparts);
}

extern "C" int lbm_step_simple(const float *g_src, float *g_dst, int nx, int ny, float tau,
                               const float *params, const lbm_fallback *fb, void *workspace,
                               size_t ws_bytes, void *stream) {
  if (int rc = check_simple("lbm_step_simple", 1, nx, ny, params)) return rc;
  if (!g_src || !g_dst) return fail(LBM_EINVAL, "lbm_step_simple: null pointer");
  if (!(tau > 0.0f)) return fail(LBM_EINVAL, "lbm_step_simple: tau must be positive");
  if (lbm::overlap(g_src, g_dst, (size_t)9 * nx * ny * sizeof(float)))
    return fail(LBM_EINVAL, "lbm_step_simple: source and destination overlap");
  if (fb && (!fb->flags || !fb->mass))
    return fail(LBM_EINVAL, "lbm_step_simple: fallback needs flags and mass pointers");
  if (!workspace || ws_bytes < simple_scratch().total)
    return fail(LBM_EWORKSPACE, "lbm_step_simple: workspace needs %zu bytes",
                simple_scratch().total);
  if (int rc = check_device()) return rc;
  hipStream_t s = (hipStream_t)stream;
  int nparts = 0;
  if (int rc = launch_simple(true, g_src, g_dst, 1, nx, ny, nullptr, tau, params, nullptr,
                             workspace, s, nparts))
    return rc;
  if (!fb) return LBM_OK;
  const SimpleScratch W = simple_scratch();
  return launch_gate(g_src, g_dst, nx, ny, tau, fb, nparts, at_(workspace, W.pmass),
                     at_(workspace, W.pflag), at_(workspace, W.pmass2),
                     at_(workspace, W.ctrl), s);
}
