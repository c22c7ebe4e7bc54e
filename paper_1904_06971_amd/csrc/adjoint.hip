// Adjoint (vector-Jacobian product) of y = A~(c) x with respect to the
// coefficient-spline control values.
#include "igs_internal.h"

extern "C" {

igs_status igs_apply_vjp(const igs_problem* pb, int32_t M, int32_t q, const double* band64, const double* x,
                         const double* ybar, double* xbar, double* cbar, void* stream) {
  (void)pb; (void)M; (void)q; (void)band64; (void)x; (void)ybar; (void)xbar; (void)cbar; (void)stream;
  return IGS_ERR_UNSUPPORTED;
}

igs_status igs_compliance_grad(const igs_problem* pb, int32_t M, int32_t q, const double* u, double* cbar,
                               void* stream) {
  (void)pb; (void)M; (void)q; (void)u; (void)cbar; (void)stream;
  return IGS_ERR_UNSUPPORTED;
}

}  // extern "C"
