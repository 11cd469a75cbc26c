// coil_coupled.h -- launchers of the fully coupled A-V solve (coil_coupled.hip).
#pragma once

#include "coil_field_fft.h"
#include "coil_field_tz.h"
#include "coil_internal.h"

namespace coilq {

// After the deferred per-wire kernels: reset the iteration, the residual of
// their solution dI_0 against the coupled system, the first preconditioned
// residual and direction.  vpub: N doubles of staging (public order).  The
// flux passes are fast convolutions when s.flux_fft (fp their plan), else
// translation-reuse passes (tp).
hipError_t launch_cg_begin(const DevState &s, const RunConst &rc, const TzPlan &tp, const FftPlan &fp, double *vpub,
                           const int *pub2int, double tol, int maxit, hipStream_t st);
// One conjugate-gradient iteration (its kernels return at once after convergence).
hipError_t launch_cg_iteration(const DevState &s, const RunConst &rc, const TzPlan &tp, const FftPlan &fp,
                               double *vpub, const int *pub2int, hipStream_t st);
// dI = dI_0 + x and the step's updates of I, q, Phi, U_w, Q_w.
hipError_t launch_cg_finish(const DevState &s, const RunConst &rc, hipStream_t st);

}  // namespace coilq
