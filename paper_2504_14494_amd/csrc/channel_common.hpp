// Walls and body force of the channel flow (the paper's Poiseuille
// validation, validation section, "Poiseuille Flow", Eq. 5): halfway
// bounce-back at the walls half a spacing outside rows 0 and ny - 1, and a
// uniform body force F = rho (gx, 0) with Guo's forcing (the velocity is
// u = (sum_i e_i f_i + F / 2) / rho, f^eq is taken at that u, and the
// collision adds (1 - omega / 2) times Guo's source).  Shared by the BGK
// channel step, the corrected channel step and its BGK fallback.
#pragma once

#include "lbm_common.hpp"

namespace lbm {

// Opposite direction: (1,3) (2,4) (5,7) (6,8).
__host__ __device__ constexpr int opp(int i) {
  return i == 0 ? 0 : (i < 5 ? (i + 1) % 4 + 1 : (i - 5 + 2) % 4 + 5);
}
static_assert(opp(1) == 3 && opp(3) == 1 && opp(2) == 4 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(7) == 5 && opp(6) == 8 && opp(8) == 6, "opp");
static_assert(cx(opp(6)) == -cx(6) && cy(opp(6)) == -cy(6), "opp");

// Pull gather with halfway bounce-back at the two walls:
// g_i(x, y) = src_i(x - cx_i, y - cy_i) when row y - cy_i lies in the
// channel, else src_opp(i)(x, y).  Opposite pairs: (1,3) (2,4) (5,7) (6,8).
template <typename T>
__device__ __forceinline__ void pull9_walls(const T *__restrict__ src, int nx, int ny, int x,
                                            int y, T (&g)[9]) {
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  const T *r0 = src + (size_t)y * 9 * nx;
  const bool below = y > 0, above = y < ny - 1;
  const T *rm = below ? r0 - (size_t)9 * nx : r0;
  const T *rp = above ? r0 + (size_t)9 * nx : r0;
  g[0] = r0[x];
  g[1] = r0[(size_t)1 * nx + xm];
  g[3] = r0[(size_t)3 * nx + xp];
  g[2] = below ? rm[(size_t)2 * nx + x] : r0[(size_t)4 * nx + x];
  g[5] = below ? rm[(size_t)5 * nx + xm] : r0[(size_t)7 * nx + x];
  g[6] = below ? rm[(size_t)6 * nx + xp] : r0[(size_t)8 * nx + x];
  g[4] = above ? rp[(size_t)4 * nx + x] : r0[(size_t)2 * nx + x];
  g[7] = above ? rp[(size_t)7 * nx + xp] : r0[(size_t)5 * nx + x];
  g[8] = above ? rp[(size_t)8 * nx + xm] : r0[(size_t)6 * nx + x];
}

// Guo's source term of direction i for the force (fx, 0) at velocity (u, v):
// w_i [3 (e_i - u) + 9 (e_i . u) e_i] . F.
template <typename T>
__device__ __forceinline__ T guo_source(int i, T fx, T u, T v) {
  const T eu = T(cx(i)) * u + T(cy(i)) * v;
  return wgt<T>(i) * fx * (T(3) * (T(cx(i)) - u) + T(9) * eu * T(cx(i)));
}

// BGK collision with Guo's body-force term, force rho * gx along x.
template <typename T>
__device__ __forceinline__ void forced_collide(T (&g)[9], T omega, T gx) {
  T drho, rho, u, v, uu;
  node_moments(g, drho, rho, u, v, uu);
  u += T(0.5) * gx;
  uu = u * u + v * v;
  const T fx = rho * gx;
  const T src_scale = T(1) - T(0.5) * omega;
#pragma unroll
  for (int i = 0; i < 9; ++i)
    g[i] = g[i] + omega * (geq_shifted<T>(i, drho, rho, u, v, uu) - g[i]) +
           src_scale * guo_source<T>(i, fx, u, v);
}

}  // namespace lbm
