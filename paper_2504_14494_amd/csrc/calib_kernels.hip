// Throughput reference for the corrected step's VALU bound.  The message
// passing rounds evaluate 1,152 GELUs per node (Methodology, "GNN
// Architecture Details": GELU after every edge message and node update), so
// their ceiling is the rate at which the VALU can evaluate the GELU sequence
// of gnn_common.hpp.  This kernel runs exactly that sequence on eight
// independent register chains per lane, with no memory traffic and no other
// work in the loop, the way copy_kernel runs the BGK step's bytes without its
// arithmetic.
#include "gnn_common.hpp"
#include "lbm_common.hpp"

namespace gnn {

constexpr int kCalibThreads = 256;
constexpr int kCalibChains = 8;

__global__ __launch_bounds__(kCalibThreads) void gelu_rate_kernel(float *__restrict__ out,
                                                                 int iters) {
  float x[kCalibChains];
#pragma unroll
  for (int j = 0; j < kCalibChains; ++j)
    x[j] = (float)(threadIdx.x & 63) * (1.0f / 32.0f) - 1.0f + 0.25f * (float)j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kCalibChains; ++j) x[j] = gelu(x[j]);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kCalibChains; ++j) s += x[j];
  out[(size_t)blockIdx.x * kCalibThreads + threadIdx.x] = s;
}

}  // namespace gnn

extern "C" int gnn_gelu_rate(float *out, int nblocks, int iters, void *stream) {
  if (!out) return lbm::fail(LBM_EINVAL, "gnn_gelu_rate: null output");
  if (nblocks < 1 || nblocks > (1 << 20) || iters < 1 || iters > (1 << 20))
    return lbm::fail(LBM_EINVAL, "gnn_gelu_rate: nblocks %d or iters %d out of range", nblocks,
                     iters);
  if (int rc = lbm::check_device()) return rc;
  hipLaunchKernelGGL(gnn::gelu_rate_kernel, dim3(nblocks), dim3(gnn::kCalibThreads), 0,
                     lbm::as_stream(stream), out, iters);
  return lbm::launch_check("gelu_rate_kernel");
}
