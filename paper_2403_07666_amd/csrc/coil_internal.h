// coil_internal.h -- device data layout and kernel launchers shared by the
// C-ABI host code (coil_api.hip) and the kernels (coil_kernels.hip).
//
// Internal element order ("wire-major"): coils concatenated; inside a coil
// wires in order w = layer*turns + turn, inside a wire the ne x ne elements in
// order a*ne + b (a radial, b axial).  A wire's elements are contiguous, so a
// 64-lane wavefront covers one wire (ne = 8) or a compact block of wires, and
// the per-wire solve reads contiguous memory.  perm[] maps internal -> public.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "coil.h"

namespace coilq {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;
// geometric mean distance of a unit square from itself, exp(<ln|p-q|>)
constexpr double kGmdSquare = 0.4470491559036625;
constexpr int kGroup = 64;       // bounding-box group = one wavefront of targets
constexpr int kMaxWireElems = 64;  // per-wire solve keeps one element per lane
constexpr int kMaxSubelements = 4;  // subelement model: subelements per wire side at most
constexpr int kFastWires = 4;       // fast wire kernel: wires (one wavefront each) per workgroup
// doubles of an n x n symmetric matrix kept as its packed lower triangle
__host__ __device__ constexpr int packed_size(int n) { return n * (n + 1) / 2; }
constexpr int kCholPad = 64;  // LDS doubles after a factorised matrix: the lanes' store sink
constexpr int kStage = 256;      // sources staged in LDS per pass
constexpr int kHT = 16;          // heat step: tile side (cells owned by a workgroup)
constexpr int kHMaxHalo = 8;     // heat step: substeps per launch at most (the tile's halo)

struct CoilDev {
    int off;        // first element (internal order)
    int n;          // elements
    int ne, ne2;    // elements per wire side, per wire
    int layers, turns;
    int wire_off;   // first wire
    int layer_off;  // first per-layer inductance block
    int group_off;  // first 64-element bounding-box group
    int nchunk;     // source chunks of the direct field pass (partial-sum slots)
    int nslot_tz;   // source-row groups of the translation-reuse pass (partial-sum slots)
    int near_base;  // mixed mode: first (target row, source row) entry of near_pair
    float c2f;      // 2 r_inner/d + 1 in grid units (FP32)
    double c2d;     // same, FP64
    double kscale;  // mu0 / (2 pi d): field per ampere in grid units
    double d;       // element side
    double dIt;     // transport-current increment per step
    double I0e;     // initial element current: the coil's I0 over the elements of a wire
    int tile_off;   // heat step: first tile of the coil
    int ntile_z;    // heat step: tiles along z
    int row_off;    // heat step: first per-row conductance record of the coil (= first grid row)
    int col_off;    // ADI heat step: first grid column of the coil
};

// heat-step conductances of one grid row (all elements of a row share them):
// faces to the rows inside and outside, axial faces, 1/V, and the border
// conductances of an inner, outer and axial border face
struct HeatRow {
    double gin, gout, gax, invV, gbin, gbout, gbax, pad;
    double ain, aout, aax;  // the face areas (ADI step: conductances from k(T))
};

struct PairItem {
    int coil, t0, tn, s0, sn, chunk;
};

// device-resident scalars
struct Scalars {
    double Q, Tpeak, sumU, maxx, Qout;
    long long step, Tpeak_pub, Tpeak_step;
    unsigned int status;
    unsigned int pad;
};

enum : unsigned { ST_NONFINITE = 1u, ST_PIVOT = 2u, ST_JC = 4u };

// device scalars of the coupled A-V solve's conjugate-gradient iteration
struct CgScalars {
    double rho, rho0, alpha, beta, tol2;
    int iters, maxit, done, pad;
};

// global constants of a run
struct RunConst {
    double Ec, n, Tc, B0, dt, dBa_dt;
    double T_bath, T_ref, C0, cp_exp;
    double u_a1;    // (p+1)/(C0 T_ref)
    double u_a0;    // (T_bath/T_ref)^(p+1)
    double u_inv;   // 1/(p+1)
    double rho_n;   // normal-state resistivity in parallel with the power law (0 = off)
    double k0, h0, k_exp, h_exp, ins_R0;  // ADI heat step: k(T), h(T), insulation between wires
    int adi;        // 1: heat step by ADI
    double em_tol;  // > 0: variable-step integration of the wire currents within a step
    int em_levels;  // finest substep dt / 2^em_levels
    float m1_near;  // mixed mode: pairs with m1 < m1_near run in FP64
    int prec;
};

// all device pointers of a handle
struct DevState {
    int N, Nw, ngroups, nitems, nheat_blocks, nsub;  // nheat_blocks: heat tiles
    int ncoils;
    int hb_slots;            // heat outflow slots per tile/line (substeps, or the ADI half steps)
    const HeatRow *hrow;     // per coil and grid row
    // ADI heat step (null otherwise)
    int adi_ncols, adi_nrows, adi_maxline;
    const double *kmult;     // thermal conductivity multiplier per element
    double *adi_Cv, *adi_G, *adi_Gbr, *adi_Gbz, *adi_Lz0, *adi_Lr1, *adi_Ts;
    const CoilDev *coils;
    const PairItem *items;
    const int4 *bbox;        // per group: min ir, max ir, min iz, max iz
    const float2 *gpos;      // (i_r, i_z) grid indices inside the coil
    const double *rho;       // radius in grid units
    const double *r, *V, *invV, *jcs, *psi;
    const double *G, *Gb;    // heat face conductances (4 per element), border
    const int *nb;           // 4 neighbours per element, -1 = border
    const int *perm;         // internal -> public index
    const int *wire_coil;    // coil of each wire
    const int *fast_w0;      // fast wire kernel: first wire of each workgroup (all of one layer)
    int nfast;               // its workgroups
    const int *elem_coil;    // coil of each element
    int max_ne2;             // largest elements-per-wire over the coils
    int tile_targets;        // field pass: targets per workgroup (= block size)
    int algo_tz;             // 1: the field partials come from the translation-reuse pass
    int algo_fft;            // 1: the field comes from the fast-convolution pass (one slot)
    int flux_fft;            // 1: the coupled solve's flux passes are fast convolutions (one slot)
    const double *Mlay;      // per layer ne2 x ne2, column-major
    const double *Minv;      // per layer inverse of Mlay, column-major
    const double *yl;        // per layer Minv * 1
    const double *syl;       // per layer sum of yl
    int *wflag;              // per wire: 1 = needs the factorising wire kernel
    const double *cw;        // per-wire Jc multiplier
    double *I, *Phi, *Br, *Bz, *E, *Ep, *dI, *q, *Jc;
    double *u[3], *T[3];     // [0] canonical state, [1], [2] heat scratch
    double2 *part;           // field partial sums: [chunk][N]
    // mixed translation pass: the kernel values near k -> 1 (FP64 evaluations
    // rounded to FP32), made once at set-up.  Pair (a, b) of a coil's rows
    // (entry near_base + a nr + b) holds g(a - b, delta) for delta = 0 .. y - 1
    // at near_val[x ..]; every |delta| < y of the pair is near, all others far.
    const int2 *near_pair;
    const float2 *near_val;
    double *Uw, *Qw, *wq, *wmaxx;
    // per-wire flux-jump / quench diagnostics: onset and quench step (-1 = not
    // yet), the wire's Joule heat before each, its max T and power density at
    // the quench step
    double *onset, *quench, *Qon, *Qqu, *Tqu, *Pqu;
    double *hb_max;          // per heat block: max T of the last substep
    long long *hb_arg;       // its public index
    double *hb_out;          // [nsub][blocks]: heat out through the borders
    Scalars *sc;
    double *tmp;             // N doubles of staging for get/set
    // coupled A-V solve (COIL_COUPLE_FULL; null otherwise)
    // subelement model: subelements per wire side (0 = one current per element)
    // and the field-driven component I_H of the element current
    int nsubel;
    double *IH;
    double *emsub;           // per wire: substeps of the last step (variable step; null otherwise)
    int cg_defer;            // 1: the per-wire kernels leave the step's updates to the coupled solve
    const double *Lself;     // ring self inductance of each element
    double *cg_x, *cg_r, *cg_z, *cg_p, *cg_q;  // correction, residual, S r, direction, A p
    double *cg_L;            // per wire: its Cholesky factor (packed lower triangle, by columns)
    double *cg_red, *cg_rw;  // per-block sums of p.q, per-wire sums of r.z
    double *cg_cw;           // per wire: the constant part moved out of the residual
    CgScalars *cg;
    // adjoint support (null in normal stepping)
    const double *src_Br, *src_Bz;    // take B^k from here instead of the field pass
    double *rec_I, *rec_Br, *rec_Bz, *rec_dI;  // record I^k, B^k, dI of the step
    double *rec_T;                    // record T at the start of each heat substep [sub][N]
};

// partial-sum slots of the last field pass (and of the transposed pass) per coil
__host__ __device__ inline int field_slots(const DevState &s, const CoilDev &c) {
    return s.algo_fft ? 1 : s.algo_tz ? c.nslot_tz : c.nchunk;
}

// ---- launchers (coil_kernels.hip) ----
hipError_t launch_field(const DevState &s, const RunConst &rc, int grid_limit, hipStream_t st);
hipError_t launch_field_finalize(const DevState &s, const RunConst &rc, hipStream_t st);
hipError_t launch_wire(const DevState &s, const RunConst &rc, hipStream_t st);
hipError_t launch_heat_step(const DevState &s, const RunConst &rc, hipStream_t st);
hipError_t launch_adi_step(const DevState &s, const RunConst &rc, hipStream_t st);
int heat_launches(int nsub);
hipError_t launch_finalize(const DevState &s, const RunConst &rc, hipStream_t st);
hipError_t launch_psi(const DevState &s, double *psi_out, hipStream_t st);
hipError_t launch_gather(const double *src, const int *perm, int n, double *dst, hipStream_t st);
hipError_t launch_scatter(const double *src, const int *perm, int n, double *dst, hipStream_t st);
hipError_t launch_u_of_T(const DevState &s, const RunConst &rc, hipStream_t st);
hipError_t launch_fill(double *p, double v, int n, hipStream_t st);
hipError_t launch_init_current(const DevState &s, hipStream_t st);
hipError_t launch_zero_int(int *p, int n, hipStream_t st);
hipError_t launch_reset_scalars(Scalars *sc, double T_bath, hipStream_t st);
hipError_t launch_stored(const DevState &s, double *out, hipStream_t st);
hipError_t launch_probe(const DevState &s, const double *zphys, int np, const double *pr, const double *pz,
                        double *br, double *bz, hipStream_t st);
// probes with the sources in nchunk chunks, partial sums in part (np * nchunk double2)
hipError_t launch_probe_chunked(const DevState &s, const double *zphys, int np, const double *pr, const double *pz,
                                double *br, double *bz, double2 *part, int nchunk, hipStream_t st);

// host-side copies of the elliptic approximations (same coefficients)
void host_ellip_f64(double m1, double *K, double *E);
void host_ellip_f32(float m1, float *K, float *E);

}  // namespace coilq
