// Stage 1 adjoint (filled in below).
#include "rpim_internal.h"

namespace rpim {

rpim_status launch_backward(rpim_plan* p, const double* X, const double* E, double nu, const double* dK, double* dE,
                            double* dX, hipStream_t s) {
  (void)p; (void)X; (void)E; (void)nu; (void)dK; (void)dE; (void)dX; (void)s;
  return RPIM_E_STATE;
}

}  // namespace rpim
