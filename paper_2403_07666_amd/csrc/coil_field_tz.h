// coil_field_tz.h -- work items and launcher of the translation-reuse field pass
// (coil_field_tz.hip).
#pragma once

#include "coil_internal.h"

namespace coilq {

// one target row segment [z0, z0 + 64 W) of row ir and a set of source rows
struct TzItem {
    int coil, ir, z0, roff, rcnt, slot, w, pad;  // source rows rows[roff .. roff + rcnt); width W
};

// per-thread target counts W = 2 .. 8; the items of one pass are ordered
// widest first and run in one launch
constexpr int kTzNW = 7;
struct TzPlan {
    const TzItem *items;
    const int *rows;  // source-row lists the items index
    int n;
    // work queue: ticket[0] forward, ticket[1] transposed pass, reset by the
    // pass's reordering kernel; grids of as many workgroups as fit at once
    int *ticket;
    int grid32, grid64, gridT32, gridT64, gridF64;
    // mixed pass input: kscale * I in public order, rounded to FP32 (made
    // with Ipub by the reordering kernel)
    float *Ipub32;
};

// resident workgroups of each field kernel on the current device (tp.grid*)
hipError_t tz_resident_grids(TzPlan &tp);

// forward pass: the currents in public order (prep), then the field kernel;
// launch_field_tz issues both
hipError_t launch_field_tz(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *Ipub,
                           const int *pub2int, int grid_limit, hipStream_t st);
hipError_t launch_field_tz_prep(const DevState &s, const TzPlan &tp, double *Ipub, hipStream_t st);
// the near kernel values of coil `coil` (rows nr), into s.near_val
hipError_t launch_near_fill(const DevState &s, int coil, int nr, hipStream_t st);
hipError_t launch_field_tz_kernel(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *Ipub,
                                  const int *pub2int, int grid_limit, hipStream_t st);

// flux pass of the coupled A-V solve: part[slot][e].y = (off-diagonal
// inductance x v)_e for v in public order (vpub); the work-queue ticket must
// have been cleared; returns at once in every workgroup when *done != 0
hipError_t launch_flux_tz(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *vpub,
                          const int *pub2int, const int *done, hipStream_t st);

// transposed pass: partT[slot][j] for the weights (wr, wz) in internal order;
// wr_pub / wz_pub are N-element staging buffers
hipError_t launch_fieldT_tz(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *wr,
                            const double *wz, double *wr_pub, double *wz_pub, const int *pub2int,
                            double *partT, hipStream_t st);

}  // namespace coilq
