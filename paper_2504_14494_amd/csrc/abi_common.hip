// Host-side error handling, device check and workspace sizing of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gnn_layout.hpp"
#include "lbm_common.hpp"

namespace lbm {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_device() {
  static int cached[64];  // 0 = unknown, 1 = ok, -1 = unsupported
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return fail(LBM_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= 64) return fail(LBM_EUNSUPPORTED, "device index %d", dev);
  if (cached[dev] == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess)
      return fail(LBM_EDEVICE, "hipGetDeviceProperties failed");
    cached[dev] = strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    if (cached[dev] < 0)
      return fail(LBM_EUNSUPPORTED, "device %d is %s, this library is built for gfx950",
                  dev, p.gcnArchName);
  }
  return cached[dev] > 0 ? LBM_OK : fail(LBM_EUNSUPPORTED, "device %d is not gfx950", dev);
}

int launch_check(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

}  // namespace lbm

extern "C" const char *lbm_last_error(void) { return lbm::g_err; }

extern "C" size_t lbm_workspace_bytes(int op, int batch, int nx, int ny, int n_rounds) {
  if (batch < 1 || nx < 1 || ny < 1) return 0;
  long long nodes = (long long)batch * nx * ny;
  switch (op) {
    case LBM_WS_MOMENTS:
    case LBM_WS_MSE:
      return (size_t)lbm::reduce_blocks(nodes) * 8 * sizeof(double);
    case LBM_WS_GNN_STEP:
      return gnn::step_workspace_bytes(nx, ny, n_rounds);
    case LBM_WS_GNN_FORWARD:
      return gnn::forward_workspace_bytes(batch, nx, ny, n_rounds);
    case LBM_WS_GNN_SAVED:
      return gnn::saved_bytes(batch, nx, ny, n_rounds);
    case LBM_WS_GNN_BACKWARD:
      return gnn::backward_workspace_bytes(batch, nx, ny, n_rounds);
    case LBM_WS_SIMPLE:
      return gnn::simple_scratch().total;
    default:
      return 0;
  }
}
