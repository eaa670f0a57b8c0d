// Channel flow between two resting walls, driven by a body force: the
// paper's Poiseuille validation (validation section, "Poiseuille Flow",
// Eq. 5: u(y) = G / (2 mu) y (H - y)).  The paper names neither a wall nor a
// forcing scheme; the ones used here are the textbook pair:
//  - halfway bounce-back: the walls lie half a spacing outside rows 0 and
//    ny - 1 (channel height H = ny); a population that would stream through
//    a wall returns to the node it left, reversed;
//  - a uniform body force F = rho (gx, 0) with Guo's forcing: the velocity is
//    u = (sum_i e_i f_i + F / 2) / rho, f^eq is taken at that u, and the
//    collision adds (1 - omega / 2) w_i [3 (e_i - u) + 9 (e_i . u) e_i] . F.
// x stays periodic.  Same storage as the periodic step: row-interleaved
// g[y][i][x] of shifted populations g = f - w; bounce-back swaps directions
// of equal weight, so it acts on g exactly as on f.
#include "channel_common.hpp"

namespace lbm {

constexpr int kChannelThreads = 256;

template <typename T>
__global__ __launch_bounds__(kChannelThreads) void channel_pull_kernel(
    const T *__restrict__ src, T *__restrict__ dst, int nx, int ny, int bx, T omega, T gx) {
  const int y = blockIdx.x / bx;
  const int x = (blockIdx.x - y * bx) * kChannelThreads + threadIdx.x;
  if (x >= nx) return;
  T g[9];
  pull9_walls(src, nx, ny, x, y, g);
  forced_collide(g, omega, gx);
  T *d = dst + (size_t)y * 9 * nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(g[i], d + (size_t)i * nx);
}

// x-average of the velocity of one row per workgroup, summed in FP64 in a
// fixed order.  The lattice holds post-collision populations, whose momentum
// already carries the whole force of the step (the forced collision adds
// rho gx), so the fluid velocity is u_x = (sum_i e_ix f*_i) / rho - gx / 2.
__global__ __launch_bounds__(kChannelThreads) void channel_profile_kernel(
    const float *__restrict__ g, int nx, float gx, double *__restrict__ prof) {
  __shared__ double red[kChannelThreads];
  const int y = blockIdx.x;
  const float *r = g + (size_t)y * 9 * nx;
  double acc = 0.0;
  for (int x = threadIdx.x; x < nx; x += kChannelThreads) {
    double f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = (double)r[(size_t)i * nx + x];
    double drho, rho, u, v, uu;
    node_moments(f, drho, rho, u, v, uu);
    acc += u - 0.5 * (double)gx;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kChannelThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) prof[y] = red[0] / (double)nx;
}

template <typename T>
static int step_channel_impl(const T *src, T *dst, int nx, int ny, T tau, T gx, void *stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "lbm_step_channel: null pointer");
  if (!lattice_ok(nx, ny)) return fail(LBM_EINVAL, "lbm_step_channel: bad lattice %d x %d", nx, ny);
  if (!(tau > T(0.5))) return fail(LBM_EINVAL, "lbm_step_channel: tau must exceed 1/2");
  if (overlap(src, dst, (size_t)9 * nx * ny * sizeof(T)))
    return fail(LBM_EINVAL, "lbm_step_channel: source and destination overlap");
  if (int rc = check_device()) return rc;
  const int bx = (nx + kChannelThreads - 1) / kChannelThreads;
  const long long blocks = (long long)bx * ny;
  if (blocks > 0x7fffffffLL) return fail(LBM_EINVAL, "lbm_step_channel: lattice too large");
  hipLaunchKernelGGL(channel_pull_kernel<T>, dim3((unsigned)blocks), dim3(kChannelThreads), 0,
                     as_stream(stream), src, dst, nx, ny, bx, T(1) / tau, gx);
  return launch_check("channel_pull_kernel");
}

}  // namespace lbm

extern "C" int lbm_step_channel(const float *g_src, float *g_dst, int nx, int ny, float tau,
                                float gx, void *stream) {
  return lbm::step_channel_impl(g_src, g_dst, nx, ny, tau, gx, stream);
}

extern "C" int lbm_step_channel_f64(const double *g_src, double *g_dst, int nx, int ny,
                                    double tau, double gx, void *stream) {
  return lbm::step_channel_impl(g_src, g_dst, nx, ny, tau, gx, stream);
}

extern "C" int lbm_channel_profile(const float *g, int nx, int ny, float gx, double *prof,
                                   void *stream) {
  if (!g || !prof) return lbm::fail(LBM_EINVAL, "lbm_channel_profile: null pointer");
  if (!lbm::lattice_ok(nx, ny))
    return lbm::fail(LBM_EINVAL, "lbm_channel_profile: bad lattice %d x %d", nx, ny);
  if (int rc = lbm::check_device()) return rc;
  hipLaunchKernelGGL(lbm::channel_profile_kernel, dim3(ny), dim3(lbm::kChannelThreads), 0,
                     lbm::as_stream(stream), g, nx, gx, prof);
  return lbm::launch_check("channel_profile_kernel");
}
