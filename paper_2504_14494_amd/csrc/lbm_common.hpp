// Shared device constants and host helpers of the gfx950 LBM-GNN library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbmgnn.h"

namespace lbm {

// D2Q9 velocity set and weights, order 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0)
// 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
__host__ __device__ constexpr int cx(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
template <typename T>
__host__ __device__ constexpr T wgt(int i) {
  return i == 0 ? T(4) / T(9) : (i < 5 ? T(1) / T(9) : T(1) / T(36));
}

// Equilibrium coefficients for the shifted form
//   g_i^eq = f_i^eq - w_i = A_i drho + rho (B_i e.u + C_i (e.u)^2 - D_i u.u)
// with A = w, B = 3w, C = 4.5w, D = 1.5w in exact arithmetic (Eq. 2 with
// c_s^2 = 1/3).  The rounded constants are chosen so that the moment
// identities hold exactly for the stored values: sum_i A_i = 1,
// sum_i B_i e_ix^2 = 1 (momentum of g^eq equals rho u, with no constant
// relative bias) and sum_i C_i e_ix^2 = sum_i D_i (mass).  With plainly
// rounded 3/9 and 3/36 the equilibrium momentum is off by a constant factor
// of about 1 + 7e-9 in FP32, which the collision feeds back every step and
// which dominates the FP32 error of long runs.
template <typename T>
struct EqCoef {
  static constexpr T A0 = T(4) / T(9);
  static constexpr T A1 = T(1) / T(9);
  static constexpr T A5 = (T(1) - A0 - T(4) * A1) / T(4);
  static constexpr T B1 = T(1) / T(3);
  static constexpr T B5 = (T(1) - T(2) * B1) / T(4);
  static constexpr T C1 = T(0.5);
  static constexpr T C5 = T(0.125);
  static constexpr T D0 = T(2) / T(3);
  static constexpr T D1 = D0 / T(4);
  static constexpr T D5 = (T(1.5) - D0 - T(4) * D1) / T(4);
  __host__ __device__ static constexpr T A(int i) { return i == 0 ? A0 : (i < 5 ? A1 : A5); }
  __host__ __device__ static constexpr T B(int i) { return i == 0 ? T(0) : (i < 5 ? B1 : B5); }
  __host__ __device__ static constexpr T C(int i) { return i == 0 ? T(0) : (i < 5 ? C1 : C5); }
  __host__ __device__ static constexpr T D(int i) { return i == 0 ? D0 : (i < 5 ? D1 : D5); }
};

// Shifted equilibrium of direction i from drho = rho - 1, rho, u, v.
template <typename T>
__host__ __device__ __forceinline__ T geq_shifted(int i, T drho, T rho, T u, T v, T uu) {
  T eu = T(cx(i)) * u + T(cy(i)) * v;
  return EqCoef<T>::A(i) * drho +
         rho * (EqCoef<T>::B(i) * eu + EqCoef<T>::C(i) * eu * eu - EqCoef<T>::D(i) * uu);
}

// Index of population i at node (x, y) of a row-interleaved lattice
// g[y][i][x] with rows of nx values.
__host__ __device__ __forceinline__ size_t pidx(int nx, int y, int i, int x) {
  return ((size_t)y * 9 + i) * (size_t)nx + x;
}

// Pull gather of one node: g_i(x, y) = src_i(x - cx_i, y - cy_i), periodic.
// `src` points at row 0 of one lattice of ny rows.
template <typename T>
__device__ __forceinline__ void pull9(const T *__restrict__ src, int nx, int ny, int x, int y,
                                      T (&g)[9]) {
  int xm = x == 0 ? nx - 1 : x - 1;
  int xp = x == nx - 1 ? 0 : x + 1;
  int ym = y == 0 ? ny - 1 : y - 1;
  int yp = y == ny - 1 ? 0 : y + 1;
  const T *r0 = src + (size_t)y * 9 * nx, *rm = src + (size_t)ym * 9 * nx,
          *rp = src + (size_t)yp * 9 * nx;
  g[0] = r0[x];
  g[1] = r0[(size_t)1 * nx + xm];
  g[2] = rm[(size_t)2 * nx + x];
  g[3] = r0[(size_t)3 * nx + xp];
  g[4] = rp[(size_t)4 * nx + x];
  g[5] = rm[(size_t)5 * nx + xm];
  g[6] = rm[(size_t)6 * nx + xp];
  g[7] = rp[(size_t)7 * nx + xp];
  g[8] = rp[(size_t)8 * nx + xm];
}

// Density deviation, density, velocity and |u|^2 of one node from its
// shifted populations (rho = 1 + sum g, rho u = sum e g).  The summation
// order pairs opposite directions so that a state at rest sums exactly.
template <typename T>
__device__ __forceinline__ void node_moments(const T (&g)[9], T &drho, T &rho, T &u, T &v,
                                             T &uu) {
  drho = ((g[0] + (g[1] + g[3])) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8]));
  T jx = (g[1] - g[3]) + ((g[5] - g[7]) + (g[8] - g[6]));
  T jy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
  rho = T(1) + drho;
  T inv = T(1) / rho;
  u = jx * inv;
  v = jy * inv;
  uu = u * u + v * v;
}

// BGK collision of one node in shifted variables (Eq. 1 with the
// equilibrium of Eq. 2).  g[] holds the pre-collision populations (already
// streamed) and is overwritten by the post-collision ones; omega = 1 / tau.
template <typename T>
__device__ __forceinline__ void bgk_collide(T (&g)[9], T omega) {
  T drho, rho, u, v, uu;
  node_moments(g, drho, rho, u, v, uu);
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = g[i] + omega * (geq_shifted<T>(i, drho, rho, u, v, uu) - g[i]);
}

// True if the byte ranges [a, a + bytes) and [b, b + bytes) intersect.
inline bool overlap(const void *a, const void *b, size_t bytes) {
  const char *p = (const char *)a, *q = (const char *)b;
  return p < q + bytes && q < p + bytes;
}

// Host-side error reporting (thread-local message, see lbm_last_error).
int fail(int code, const char *fmt, ...);
// Checks that the current device is gfx950 (cached per device).
int check_device();
// Maps the last HIP launch error to LBM_EDEVICE.
int launch_check(const char *what);

inline bool lattice_ok(int nx, int ny) {
  return nx >= 1 && ny >= 1 && (long long)nx * ny < (1LL << 31);
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Number of bytes a reduction over `nodes` items leaves as FP64 partials.
constexpr int kReduceThreads = 256;
constexpr int kReduceMaxBlocks = 1024;
inline int reduce_blocks(long long nodes) {
  long long b = (nodes + kReduceThreads - 1) / kReduceThreads;
  if (b < 1) b = 1;
  return b > kReduceMaxBlocks ? kReduceMaxBlocks : (int)b;
}

}  // namespace lbm
