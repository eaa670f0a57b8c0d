// D2Q9 lattice Boltzmann kernels for gfx950: equilibrium initialisation,
// the fused pull-scheme BGK step (Eq. 1 with the equilibrium of Eq. 2),
// moments with FP64 observables, and the fine-to-coarse restriction used to
// build training data.
//
// Storage: g_i = f_i - w_i in row-interleaved structure-of-arrays form,
// g[y][i][x]: each lattice row holds nine contiguous runs of nx values, one
// per direction.  Storing the deviation from the rest weights keeps the FP32
// roundoff of the density sum at the level of the flow signal instead of the
// O(1) weights.  Keeping the nine directions of a row together means that
// the eighteen load and store streams of a step all fall inside a window of
// three rows (27 nx values) instead of nine planes that are whole lattices
// apart, which keeps HBM pages and channels busy evenly.
#include <cstdlib>

#include "lbm_common.hpp"

namespace lbm {

// ------------------------------------------------------------------ init ---

template <typename T>
__global__ void init_kernel(T *__restrict__ g, int nx, int ny, const T *__restrict__ rho,
                            const T *__restrict__ ux, const T *__restrict__ uy) {
  size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (size_t)nx * ny) return;
  int x = (int)(n % nx), y = (int)(n / nx);
  T r = rho[n], u = ux[n], v = uy[n];
  T uu = u * u + v * v;
#pragma unroll
  for (int i = 0; i < 9; ++i) g[pidx(nx, y, i, x)] = geq_shifted<T>(i, r - T(1), r, u, v, uu);
}

// Post-collision image of the first-order Chapman-Enskog state: the
// pre-collision state f^eq - (tau w_i rho / c_s^2) Q_i : S (Q_i = e_i e_i -
// c_s^2 I, S the symmetric velocity gradient by second-order central
// differences, periodic) after one BGK collision, which scales its
// non-equilibrium part by 1 - 1/tau: f^eq - ((tau - 1) w_i rho / c_s^2) Q_i : S.
// A state on the slow manifold: it does not excite the period-2 mode that a
// pure equilibrium start launches.
template <typename T>
__global__ void init_ce_kernel(T *__restrict__ g, int nx, int ny, const T *__restrict__ rho,
                               const T *__restrict__ ux, const T *__restrict__ uy, T tau) {
  size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (size_t)nx * ny) return;
  int x = (int)(n % nx), y = (int)(n / nx);
  size_t row = (size_t)y * nx;
  size_t xp = row + (x + 1 == nx ? 0 : x + 1), xm = row + (x == 0 ? nx - 1 : x - 1);
  size_t yp = (size_t)(y + 1 == ny ? 0 : y + 1) * nx + x;
  size_t ym = (size_t)(y == 0 ? ny - 1 : y - 1) * nx + x;
  T sxx = T(0.5) * (ux[xp] - ux[xm]);
  T syy = T(0.5) * (uy[yp] - uy[ym]);
  T sxy = T(0.25) * ((ux[yp] - ux[ym]) + (uy[xp] - uy[xm]));
  T r = rho[n], u = ux[n], v = uy[n];
  T uu = u * u + v * v;
  const T cs2 = T(1) / T(3);
  T pre = (tau - T(1)) * r / cs2;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    T qs = (T(cx(i) * cx(i)) - cs2) * sxx + T(2 * cx(i) * cy(i)) * sxy +
           (T(cy(i) * cy(i)) - cs2) * syy;
    g[pidx(nx, y, i, x)] = geq_shifted<T>(i, r - T(1), r, u, v, uu) - pre * wgt<T>(i) * qs;
  }
}

// ------------------------------------------------------------ BGK, fused ---

constexpr int kBgkThreads = 256;

// One thread per node.  The grid is one-dimensional: block b covers
// kBgkThreads consecutive x of row b / bx, bx = ceil(nx / kBgkThreads).
// Consecutive blocks walk along a row, so blocks that share an x range in
// neighbouring rows (and hence the rows they pull from) are issued bx apart;
// when bx is a multiple of the 8 XCDs they land on the same XCD and its L2.
template <typename T>
__global__ __launch_bounds__(kBgkThreads) void bgk_pull_kernel(const T *__restrict__ src,
                                                               T *__restrict__ dst, int nx,
                                                               int ny, int bx, T omega) {
  int y = blockIdx.x / bx;
  int x = (blockIdx.x - y * bx) * kBgkThreads + threadIdx.x;
  if (x >= nx) return;
  T g[9];
  pull9(src, nx, ny, x, y, g);
  bgk_collide(g, omega);
  T *d = dst + (size_t)y * 9 * nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(g[i], d + (size_t)i * nx);
}

// Lane l of a wave takes lane l - 1's v (the value at x - 1), lane 0 takes
// `halo` (DPP wave_shr:1).
__device__ __forceinline__ float wave_from_left(float v, float halo) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, halo),
                                                               __builtin_bit_cast(int, v), 0x138,
                                                               0xF, 0xF, false));
}
// Lane l takes lane l + 1's v (the value at x + 1), lane 63 takes `halo`
// (DPP wave_shl:1).
__device__ __forceinline__ float wave_from_right(float v, float halo) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, halo),
                                                               __builtin_bit_cast(int, v), 0x130,
                                                               0xF, 0xF, false));
}

// The same step in FP32, by waves of 64 consecutive nodes of a row.  The
// six populations that move along x are not gathered from x -/+ 1: every
// lane loads its own column, so each of the nine loads of a wave covers two
// whole 128-byte lines, and the values move one lane over through DPP.  The
// two columns just outside the wave (x0 - 1 and x0 + 64, periodic) are
// wave-uniform addresses, fetched by scalar loads, so the vector memory path
// sees exactly the 18 lines of the wave.  Cache policy, measured on
// back-to-back steps: the three populations that do not move along x are
// read once by one wave and bypass the caches (non-temporal); the six that
// move keep normal loads, because their edge lines are read again, as a
// halo, by the neighbouring wave (non-temporal there costs a second HBM
// fetch of those lines).  A row's last wave, when nx is not a multiple of
// 64, is partial and uses the per-lane gather of bgk_pull_kernel instead.
// Same arithmetic, bitwise the same result as bgk_pull_kernel, about 3%
// faster at 4096^2 and 8192^2.
__global__ __launch_bounds__(kBgkThreads) void bgk_pull_wave_kernel(
    const float *__restrict__ src, float *__restrict__ dst, int nx, int ny, int bx,
    float omega) {
  const int y = blockIdx.x / bx;
  const int lane = threadIdx.x & 63;
  const int x0 = __builtin_amdgcn_readfirstlane((blockIdx.x - y * bx) * kBgkThreads +
                                                (threadIdx.x & ~63));
  if (x0 >= nx) return;
  const int x = x0 + lane;
  if (x0 + 64 > nx) {
    // the row's last wave is partial: the per-lane gather (no lane shifts)
    if (x >= nx) return;
    float g[9];
    pull9(src, nx, ny, x, y, g);
    bgk_collide(g, omega);
    float *d = dst + (size_t)y * 9 * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(g[i], d + (size_t)i * nx);
    return;
  }
  // from here every lane of the wave is active, as the lane shifts need
  const int xl = x0 == 0 ? nx - 1 : x0 - 1;
  const int xr = x0 + 64 == nx ? 0 : x0 + 64;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const float *r0 = src + (size_t)y * 9 * nx, *rm = src + (size_t)ym * 9 * nx,
              *rp = src + (size_t)yp * 9 * nx;
  const float h1 = r0[(size_t)1 * nx + xl], h5 = rm[(size_t)5 * nx + xl],
              h8 = rp[(size_t)8 * nx + xl];
  const float h3 = r0[(size_t)3 * nx + xr], h6 = rm[(size_t)6 * nx + xr],
              h7 = rp[(size_t)7 * nx + xr];
  const float a1 = r0[(size_t)1 * nx + x], a5 = rm[(size_t)5 * nx + x],
              a8 = rp[(size_t)8 * nx + x];
  const float a3 = r0[(size_t)3 * nx + x], a6 = rm[(size_t)6 * nx + x],
              a7 = rp[(size_t)7 * nx + x];
  float g[9];
  g[0] = __builtin_nontemporal_load(r0 + x);
  g[2] = __builtin_nontemporal_load(rm + (size_t)2 * nx + x);
  g[4] = __builtin_nontemporal_load(rp + (size_t)4 * nx + x);
  g[1] = wave_from_left(a1, h1);
  g[5] = wave_from_left(a5, h5);
  g[8] = wave_from_left(a8, h8);
  g[3] = wave_from_right(a3, h3);
  g[6] = wave_from_right(a6, h6);
  g[7] = wave_from_right(a7, h7);
  bgk_collide(g, omega);
  float *d = dst + (size_t)y * 9 * nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(g[i], d + (size_t)i * nx);
}

template <typename T>
int launch_bgk(const T *src, T *dst, int nx, int ny, T tau, hipStream_t s) {
  int bx = (nx + kBgkThreads - 1) / kBgkThreads;
  long long blocks = (long long)bx * ny;
  if (blocks > 0x7fffffffLL) return fail(LBM_EINVAL, "lbm_step_bgk: lattice too large");
  if constexpr (sizeof(T) == sizeof(float)) {
    hipLaunchKernelGGL(bgk_pull_wave_kernel, dim3((unsigned)blocks), dim3(kBgkThreads), 0, s,
                       src, dst, nx, ny, bx, T(1) / tau);
    return launch_check("bgk_pull_wave_kernel");
  }
  hipLaunchKernelGGL(bgk_pull_kernel<T>, dim3((unsigned)blocks), dim3(kBgkThreads), 0, s, src,
                     dst, nx, ny, bx, T(1) / tau);
  return launch_check("bgk_pull_kernel");
}

// Streaming alone (the left-hand side of Eq. 1): dst_i(x) = src_i(x - e_i).
template <typename T>
__global__ __launch_bounds__(kBgkThreads) void stream_kernel(const T *__restrict__ src,
                                                             T *__restrict__ dst, int nx, int ny,
                                                             int bx) {
  int y = blockIdx.x / bx;
  int x = (blockIdx.x - y * bx) * kBgkThreads + threadIdx.x;
  if (x >= nx) return;
  T g[9];
  pull9(src, nx, ny, x, y, g);
  T *d = dst + (size_t)y * 9 * nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) d[(size_t)i * nx] = g[i];
}

// ----------------------------------------------------- moments + sums ---

__device__ __forceinline__ void tgv_field(const lbm_tgv &a, int x, int y, double &ux,
                                          double &uy) {
  double d = exp(-a.nu * (a.kx * a.kx + a.ky * a.ky) * a.t);
  double X = x - a.x0, Y = y - a.y0;
  double sx, cxv, sy, cyv;
  sincos(a.kx * X, &sx, &cxv);
  sincos(a.ky * Y, &sy, &cyv);
  ux = -a.u0 * cxv * sy * d;
  uy = a.u0 * (a.kx / a.ky) * sx * cyv * d;
}

// Fixed-order block reduction of 8 doubles; slot 6 is a minimum.
__device__ void block_reduce8(double (&acc)[8], double *out) {
  __shared__ double sh[8][kReduceThreads];
  int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[k][t] = acc[k];
  __syncthreads();
  for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        sh[k][t] = k == 6 ? fmin(sh[k][t], sh[k][t + s]) : sh[k][t] + sh[k][t + s];
    }
    __syncthreads();
  }
  if (t < 8) out[t] = sh[t][0];
}

__global__ __launch_bounds__(kReduceThreads) void moments_kernel(
    const float *__restrict__ g, int nx, int ny, float *__restrict__ rho_out,
    float *__restrict__ ux_out, float *__restrict__ uy_out, lbm_tgv a, int with_tgv,
    double *__restrict__ partials) {
  size_t nodes = (size_t)nx * ny;
  double acc[8] = {0, 0, 0, 0, 0, 0, INFINITY, 0};
  for (size_t n = (size_t)blockIdx.x * kReduceThreads + threadIdx.x; n < nodes;
       n += (size_t)gridDim.x * kReduceThreads) {
    int x = (int)(n % nx), y = (int)(n / nx);
    double f[9];
    double drho = 0, jx = 0, jy = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double gi = (double)g[pidx(nx, y, i, x)];
      f[i] = gi + wgt<double>(i);
      drho += gi;
      jx += cx(i) * gi;
      jy += cy(i) * gi;
    }
    double rho = 1.0 + drho;
    double u = jx / rho, v = jy / rho;
    if (rho_out) rho_out[n] = (float)rho;
    if (ux_out) ux_out[n] = (float)u;
    if (uy_out) uy_out[n] = (float)v;
    acc[0] += drho;  // total mass = nodes + sum(drho), added at the end
    acc[1] += jx;
    acc[2] += jy;
    acc[3] += 0.5 * (u * u + v * v);
    if (with_tgv) {
      double uax, uay;
      tgv_field(a, x, y, uax, uay);
      acc[4] += (u - uax) * (u - uax) + (v - uay) * (v - uay);
      acc[5] += uax * uax + uay * uay;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      acc[6] = fmin(acc[6], f[i]);
      acc[7] += f[i] < 0.0 ? 1.0 : 0.0;
    }
  }
  block_reduce8(acc, partials + (size_t)blockIdx.x * 8);
}

__global__ __launch_bounds__(kReduceThreads) void moments_finalize(
    const double *__restrict__ partials, int nblocks, double nodes, double *__restrict__ sums) {
  double acc[8] = {0, 0, 0, 0, 0, 0, INFINITY, 0};
  for (int b = threadIdx.x; b < nblocks; b += kReduceThreads) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      acc[k] = k == 6 ? fmin(acc[k], partials[b * 8 + k]) : acc[k] + partials[b * 8 + k];
  }
  __shared__ double out[8];
  block_reduce8(acc, out);
  __syncthreads();
  if (threadIdx.x < 8) sums[threadIdx.x] = threadIdx.x == 0 ? nodes + out[0] : out[threadIdx.x];
}

// ------------------------------------------------------------ restriction ---

// Fine and coarse lattices are both row-interleaved.  One thread per coarse
// population value.
__global__ void restrict_kernel(const double *__restrict__ gf, int nxf, int nyf, int factor,
                                double lambda, int pull, int unstream,
                                float *__restrict__ gc) {
  int nxc = nxf / factor, nyc = nyf / factor;
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)9 * nxc * nyc) return;
  // idx = (Yo * 9 + i) * nxc + Xo
  int Xo = (int)(idx % nxc);
  size_t rest = idx / nxc;
  int i = (int)(rest % 9), Yo = (int)(rest / 9);
  int X = Xo, Y = Yo;
  if (unstream) {  // out_i(X) = R_i(X + e_i)
    X = (X + cx(i) + nxc) % nxc;
    Y = (Y + cy(i) + nyc) % nyc;
  }
  int xf = X * factor, yf = Y * factor;
  double f[9], rho = 0, jx = 0, jy = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    int xs = xf, ys = yf;
    if (pull) {
      xs = (xf - cx(k) + nxf) % nxf;
      ys = (yf - cy(k) + nyf) % nyf;
    }
    f[k] = gf[pidx(nxf, ys, k, xs)] + wgt<double>(k);
    rho += f[k];
    jx += cx(k) * f[k];
    jy += cy(k) * f[k];
  }
  double u = jx / rho, v = jy / rho, usq = 1.5 * (u * u + v * v);
  double pxx = 0, pxy = 0, pyy = 0, feq_i = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double eu = cx(k) * u + cy(k) * v;
    double feq = wgt<double>(k) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - usq);
    double d = f[k] - feq;
    pxx += cx(k) * cx(k) * d;
    pxy += cx(k) * cy(k) * d;
    pyy += cy(k) * cy(k) * d;
    if (k == i) feq_i = feq;
  }
  const double cs2 = 1.0 / 3.0;
  double qxx = cx(i) * cx(i) - cs2, qyy = cy(i) * cy(i) - cs2, qxy = cx(i) * cy(i);
  double fneq = wgt<double>(i) / (2.0 * cs2 * cs2) * (qxx * pxx + 2.0 * qxy * pxy + qyy * pyy);
  double fc = feq_i + lambda * fneq;
  gc[idx] = (float)(fc - wgt<double>(i));
}

// ------------------------------------------------------------------ copy ---

typedef float vf4 __attribute__((ext_vector_type(4)));

// One 16-byte element per thread, non-temporal loads and stores: the plain
// streaming copy that bounds what a read-once write-once kernel can reach.
// (Measured at 8192^2 x 9 floats: 6.56 TB/s; with cached loads 6.26 TB/s, and
// with 2, 4 or 8 elements per thread or 512-1024 threads per block, slower.)
__global__ __launch_bounds__(256) void copy_kernel(const vf4 *__restrict__ src,
                                                   vf4 *__restrict__ dst, size_t n4) {
  size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[k]), &dst[k]);
}

__global__ void copy_tail_kernel(const float *__restrict__ src, float *__restrict__ dst,
                                 size_t from, size_t n) {
  size_t k = from + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k];
}

}  // namespace lbm

using namespace lbm;

// ------------------------------------------------------------------- ABI ---

template <typename T>
static int init_impl(T *g, int nx, int ny, const T *rho, const T *ux, const T *uy,
                     void *stream) {
  if (!g || !rho || !ux || !uy) return fail(LBM_EINVAL, "lbm_init: null pointer");
  if (!lattice_ok(nx, ny)) return fail(LBM_EINVAL, "lbm_init: bad lattice %d x %d", nx, ny);
  if (int rc = check_device()) return rc;
  size_t nodes = (size_t)nx * ny;
  hipLaunchKernelGGL(init_kernel<T>, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0,
                     as_stream(stream), g, nx, ny, rho, ux, uy);
  return launch_check("init_kernel");
}

template <typename T>
static int init_ce_impl(T *g, int nx, int ny, const T *rho, const T *ux, const T *uy, T tau,
                        void *stream) {
  if (!g || !rho || !ux || !uy) return fail(LBM_EINVAL, "lbm_init_ce: null pointer");
  if (!lattice_ok(nx, ny)) return fail(LBM_EINVAL, "lbm_init_ce: bad lattice %d x %d", nx, ny);
  if (!(tau > T(0))) return fail(LBM_EINVAL, "lbm_init_ce: tau must be positive");
  if (int rc = check_device()) return rc;
  size_t nodes = (size_t)nx * ny;
  hipLaunchKernelGGL(init_ce_kernel<T>, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0,
                     as_stream(stream), g, nx, ny, rho, ux, uy, tau);
  return launch_check("init_ce_kernel");
}

extern "C" int lbm_init_ce(float *g, int nx, int ny, const float *rho, const float *ux,
                           const float *uy, float tau, void *stream) {
  return init_ce_impl(g, nx, ny, rho, ux, uy, tau, stream);
}

extern "C" int lbm_init_ce_f64(double *g, int nx, int ny, const double *rho, const double *ux,
                               const double *uy, double tau, void *stream) {
  return init_ce_impl(g, nx, ny, rho, ux, uy, tau, stream);
}

extern "C" int lbm_init(float *g, int nx, int ny, const float *rho, const float *ux,
                        const float *uy, void *stream) {
  return init_impl(g, nx, ny, rho, ux, uy, stream);
}

extern "C" int lbm_init_f64(double *g, int nx, int ny, const double *rho, const double *ux,
                            const double *uy, void *stream) {
  return init_impl(g, nx, ny, rho, ux, uy, stream);
}

template <typename T>
static int step_bgk_impl(const T *src, T *dst, int nx, int ny, T tau, void *stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "lbm_step_bgk: null pointer");
  if (!lattice_ok(nx, ny)) return fail(LBM_EINVAL, "lbm_step_bgk: bad lattice %d x %d", nx, ny);
  if (!(tau > T(0))) return fail(LBM_EINVAL, "lbm_step_bgk: tau must be positive");
  size_t bytes = (size_t)9 * nx * ny * sizeof(T);
  if (overlap(src, dst, bytes))
    return fail(LBM_EINVAL, "lbm_step_bgk: source and destination overlap");
  if (int rc = check_device()) return rc;
  return launch_bgk(src, dst, nx, ny, tau, as_stream(stream));
}

extern "C" int lbm_step_bgk(const float *g_src, float *g_dst, int nx, int ny, float tau,
                            void *stream) {
  return step_bgk_impl(g_src, g_dst, nx, ny, tau, stream);
}

extern "C" int lbm_step_bgk_f64(const double *g_src, double *g_dst, int nx, int ny,
                                double tau, void *stream) {
  return step_bgk_impl(g_src, g_dst, nx, ny, tau, stream);
}

extern "C" int lbm_stream(const float *g_src, float *g_dst, int nx, int ny, int batch,
                          void *stream) {
  if (!g_src || !g_dst) return fail(LBM_EINVAL, "lbm_stream: null pointer");
  if (batch < 1 || !lattice_ok(nx, ny) || (long long)batch * nx * ny >= (1LL << 31))
    return fail(LBM_EINVAL, "lbm_stream: bad sizes");
  size_t per = (size_t)9 * nx * ny;
  if (overlap(g_src, g_dst, per * batch * sizeof(float)))
    return fail(LBM_EINVAL, "lbm_stream: source and destination overlap");
  if (int rc = check_device()) return rc;
  int bx = (nx + kBgkThreads - 1) / kBgkThreads;
  long long blocks = (long long)bx * ny;
  if (blocks > 0x7fffffffLL) return fail(LBM_EINVAL, "lbm_stream: lattice too large");
  for (int b = 0; b < batch; ++b) {
    hipLaunchKernelGGL(stream_kernel<float>, dim3((unsigned)blocks), dim3(kBgkThreads), 0,
                       as_stream(stream), g_src + b * per, g_dst + b * per, nx, ny, bx);
    if (int rc = launch_check("stream_kernel")) return rc;
  }
  return LBM_OK;
}

extern "C" int lbm_moments(const float *g, int nx, int ny, float *rho, float *ux, float *uy,
                           const lbm_tgv *analytic, double *sums, void *workspace,
                           size_t ws_bytes, void *stream) {
  if (!g) return fail(LBM_EINVAL, "lbm_moments: null populations");
  if (!lattice_ok(nx, ny)) return fail(LBM_EINVAL, "lbm_moments: bad lattice %d x %d", nx, ny);
  if (!sums && !rho && !ux && !uy) return LBM_OK;
  long long nodes = (long long)nx * ny;
  int nb = reduce_blocks(nodes);
  size_t need = (size_t)nb * 8 * sizeof(double);
  if (!workspace || ws_bytes < need)
    return fail(LBM_EWORKSPACE, "lbm_moments: workspace needs %zu bytes", need);
  if (analytic && !(analytic->ky != 0.0))
    return fail(LBM_EINVAL, "lbm_moments: analytic field needs ky != 0");
  if (int rc = check_device()) return rc;
  lbm_tgv a{};
  int with = 0;
  if (analytic) {
    a = *analytic;
    with = 1;
  }
  hipStream_t s = as_stream(stream);
  double *part = (double *)workspace;
  hipLaunchKernelGGL(moments_kernel, dim3(nb), dim3(kReduceThreads), 0, s, g, nx, ny, rho, ux,
                     uy, a, with, part);
  if (int rc = launch_check("moments_kernel")) return rc;
  if (sums) {
    hipLaunchKernelGGL(moments_finalize, dim3(1), dim3(kReduceThreads), 0, s, part, nb,
                       (double)nodes, sums);
    return launch_check("moments_finalize");
  }
  return LBM_OK;
}

extern "C" int lbm_restrict(const double *g_fine, int nxf, int nyf, int factor, double tau_f,
                            double tau_c, int pull, int unstream, float *g_coarse,
                            void *stream) {
  if (!g_fine || !g_coarse) return fail(LBM_EINVAL, "lbm_restrict: null pointer");
  if (factor < 1 || !lattice_ok(nxf, nyf) || nxf % factor || nyf % factor)
    return fail(LBM_EINVAL, "lbm_restrict: %d x %d is not a multiple of %d", nxf, nyf, factor);
  if (!(tau_f > 0) || !(tau_c > 0)) return fail(LBM_EINVAL, "lbm_restrict: tau must be > 0");
  if (int rc = check_device()) return rc;
  size_t n = (size_t)9 * (nxf / factor) * (nyf / factor);
  hipLaunchKernelGGL(restrict_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     as_stream(stream), g_fine, nxf, nyf, factor, factor * tau_c / tau_f,
                     pull, unstream, g_coarse);
  return launch_check("restrict_kernel");
}

extern "C" int lbm_copy(const float *src, float *dst, size_t n, void *stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "lbm_copy: null pointer");
  if (((uintptr_t)src | (uintptr_t)dst) & 15)
    return fail(LBM_EINVAL, "lbm_copy: pointers must be 16-byte aligned");
  if (overlap(src, dst, n * sizeof(float)))
    return fail(LBM_EINVAL, "lbm_copy: source and destination overlap");
  if (int rc = check_device()) return rc;
  hipStream_t s = as_stream(stream);
  size_t n4 = n / 4;
  if (n4) {
    size_t blocks = (n4 + 255) / 256;
    if (blocks > 0x7fffffffULL) return fail(LBM_EINVAL, "lbm_copy: too large");
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const vf4 *)src, (vf4 *)dst, n4);
    if (int rc = launch_check("copy_kernel")) return rc;
  }
  if (n4 * 4 < n) {
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(64), 0, s, src, dst, n4 * 4, n);
    return launch_check("copy_tail_kernel");
  }
  return LBM_OK;
}
