// GNN-corrected collision (placeholder entry points until the kernels land).
#include "gnn_layout.hpp"
#include "lbm_common.hpp"

using namespace lbm;

extern "C" size_t gnn_param_count(int n_rounds) {
  if (n_rounds < 1 || n_rounds > gnn::MAX_ROUNDS) return 0;
  return gnn::blob_layout(n_rounds).nparam;
}
extern "C" size_t gnn_blob_len(int n_rounds) {
  if (n_rounds < 1 || n_rounds > gnn::MAX_ROUNDS) return 0;
  return gnn::blob_layout(n_rounds).total;
}
extern "C" int lbm_step_gnn(const float *, float *, int, int, float, const float *, int,
                            const lbm_fallback *, void *, size_t, void *) {
  return fail(LBM_EUNSUPPORTED, "lbm_step_gnn: not built yet");
}
extern "C" int gnn_forward(const float *, float *, int, int, int, const float *, const float *,
                           int, float *, void *, size_t, void *, size_t, void *) {
  return fail(LBM_EUNSUPPORTED, "gnn_forward: not built yet");
}
extern "C" int gnn_backward(const float *, const float *, const void *, int, int, int,
                            const float *, const float *, int, float *, void *, size_t, void *) {
  return fail(LBM_EUNSUPPORTED, "gnn_backward: not built yet");
}
extern "C" int gnn_mse(const float *, const float *, int, int, int, double, double *, float *,
                       void *, size_t, void *) {
  return fail(LBM_EUNSUPPORTED, "gnn_mse: not built yet");
}
extern "C" int gnn_adam(float *, const float *, float *, float *, size_t, float, float, float,
                        float, int, void *) {
  return fail(LBM_EUNSUPPORTED, "gnn_adam: not built yet");
}
