// Shape sensitivities of u^T K u (Section 4.1.2).
#include "device_common.h"

using namespace igamt;

extern "C" igamt_status igamt_grad_workspace_bytes(const igamt_plan *P, igamt_precision prec, int64_t *bytes) {
  set_error("not implemented");
  return IGAMT_EUNSUPPORTED;
}

extern "C" igamt_status igamt_uKu_grad(igamt_plan *P, double E, double nu, igamt_precision prec, const double *d_u,
                                       double *d_grad, double *d_uKu, void *d_workspace, void *stream) {
  set_error("not implemented");
  return IGAMT_EUNSUPPORTED;
}
