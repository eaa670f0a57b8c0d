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
