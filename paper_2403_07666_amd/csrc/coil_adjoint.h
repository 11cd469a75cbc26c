// coil_adjoint.h -- adjoint kernel arguments and launchers (coil_adjoint.hip).
#pragma once

#include "coil_internal.h"

namespace coilq {

// per-step pointers of the reverse wire kernel (internal element order)
struct AdjPtrs {
    const double *I, *T, *Br, *Bz, *dI;  // forward I^k, T^k, B^k, dI of step k
    const double *qbar;                  // adjoint of the step's Joule source
    double *Ibar;                        // in: adjoint of I^{k+1}; out: of I^k (without G^T Bbar)
    double *ubar;                        // adjoint of u^k (+= T'(u) Tbar)
    double *wr, *wz;                     // out: field-transpose weights
    double *cbar, *dItbar;               // per wire, accumulated over steps
};

hipError_t launch_fieldT(const DevState &s, const RunConst &rc, int grid_limit, const double *wr,
                         const double *wz, double *partT, hipStream_t st);
hipError_t launch_fieldT_sum(const DevState &s, const double *partT, double *out, int accumulate,
                             hipStream_t st);
hipError_t launch_field_weights(const DevState &s, double *br, double *bz, hipStream_t st);
hipError_t launch_wire_adj(const DevState &s, const RunConst &rc, const AdjPtrs &a, hipStream_t st);
hipError_t launch_heat_adj(const DevState &s, const RunConst &rc, const double *ub_in, double *ub_out,
                           const double *Tsub, double *qbar, hipStream_t st);
hipError_t launch_qbar_init(const DevState &s, double *qbar, double wQdt, hipStream_t st);
hipError_t launch_add_at(double *p, int i, double v, hipStream_t st);
hipError_t launch_set_step(Scalars *sc, long long step, hipStream_t st);
hipError_t launch_copy(const double *src, double *dst, int n, hipStream_t st);

}  // namespace coilq
