// Learned lookup tables: POD basis and MLP kernels.
#include "device_common.h"

using namespace igamt;

extern "C" igamt_status igamt_pod_build(const double *d_snap, int32_t n_s, int64_t n_e, int32_t r, float *d_mean,
                                        float *d_basis, double *h_sigma, double *d_work, void *stream) {
  set_error("not implemented"); return IGAMT_EUNSUPPORTED;
}
extern "C" igamt_status igamt_table_from_pod(igamt_plan *P, const float *d_mean, const float *d_basis, int32_t r,
                                             const float *d_coeffs, void *stream) {
  set_error("not implemented"); return IGAMT_EUNSUPPORTED;
}
extern "C" igamt_status igamt_table_rows_error(const igamt_plan *P, const int32_t *d_rows, int32_t n_rows,
                                               const double *d_exact, double *d_err, void *stream) {
  set_error("not implemented"); return IGAMT_EUNSUPPORTED;
}
extern "C" int64_t igamt_mlp_n_params(const igamt_mlp_desc *desc) { return 0; }
extern "C" igamt_status igamt_mlp_forward(const igamt_mlp_desc *desc, const float *d_params, const float *d_x,
                                          float *d_act, float *d_y, void *stream) {
  set_error("not implemented"); return IGAMT_EUNSUPPORTED;
}
extern "C" igamt_status igamt_mse_loss(const igamt_mlp_desc *desc, const float *d_y, const float *d_target,
                                       float *d_dy, float *d_loss, void *stream) {
  set_error("not implemented"); return IGAMT_EUNSUPPORTED;
}
extern "C" igamt_status igamt_mlp_backward(const igamt_mlp_desc *desc, const float *d_params, const float *d_x,
                                           const float *d_act, const float *d_dy, float *d_grads, float *d_scratch,
                                           void *stream) {
  set_error("not implemented"); return IGAMT_EUNSUPPORTED;
}
extern "C" igamt_status igamt_adam_step(float *d_params, const float *d_grads, float *d_m, float *d_v, int64_t n,
                                        float lr, float beta1, float beta2, float eps, int32_t step, void *stream) {
  set_error("not implemented"); return IGAMT_EUNSUPPORTED;
}
