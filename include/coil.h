/*
 * coil.h -- C ABI of the MI355X (gfx950) coil quench hot path.
 *
 * What the library computes (Xue et al., "Holistic numerical simulation of a
 * quenching process on a real-size multifilamentary superconducting coil";
 * Methods: "Numerical Algorithm", the heat-diffusion paragraph and the E-J
 * paragraph; Fig. 1(b) and Fig. 2(a,b)):
 *   the (r,z) cross-section of one or more solenoids, each wire split into
 *   ne x ne square current elements treated as coaxial rings.  One time step:
 *     1. all-pairs field sum B_e = B_a(t) z + sum_{j != e} G_B(e,j) I_j with the
 *        coaxial-ring Green's function (complete elliptic integrals K, E
 *        evaluated on the fly);
 *     2. local power law E = Ec (|J|/Jc)^n sgn J, Jc = c_w Jc0 mu_e (1 - T/Tc)
 *        B0/(B0 + |B|) (1 - eps_coef |eps|^eps_pow), from the state at step k
 *        (optionally in parallel with a normal-state resistivity rho_n, so that
 *        the flux-flow and normal states of a quench are covered);
 *     3. per-wire A-V solve: each wire's element currents respond to the flux
 *        of the other wires' transport current and of the background field,
 *        one loop voltage per wire enforces the wire's transport current
 *        (linearised backward Euler);
 *     4. explicit heat step c dT/dt = div(k grad T) + E.J on the enthalpy, with
 *        a Robin condition h (T - T_bath) on the four borders, sub-cycled;
 *     5. reductions: Joule heat Q (total and per wire), peak temperature,
 *        terminal voltage, max |J|/Jc.
 *
 * Conventions
 *   - Every function returns int: COIL_OK (0) or a negative COIL_E_* code;
 *     coil_last_error() then holds a message (thread-local).  No C++ exception
 *     crosses the ABI.  Arguments are validated before any allocation or
 *     launch.
 *   - Units: SI (m, s, A, T, V, K, J).
 *   - Element order seen through this ABI ("public order"): coils concatenated;
 *     inside a coil the (r,z) grid is row-major, e = i_r * n_z + i_z, with
 *     n_r = layers*ne radial and n_z = turns*ne axial elements, i_r = 0 at
 *     r_inner and i_z = 0 at the bottom.  Wire order: w = layer*turns + turn,
 *     coils concatenated.  The internal device layout is the library's own.
 *   - Device memory: the caller owns one device workspace (e.g. a torch uint8
 *     tensor) of the size coil_query() reports and keeps it alive until
 *     coil_destroy().  The library allocates no device memory of its own
 *     except where a function says so.
 *   - Streams: every call enqueues on the HIP stream given to coil_init
 *     (coil_run may fork work to a second stream of the handle's own, which
 *     it joins back into that stream before returning).  Only
 *     coil_run at report points, coil_scalars, host-destination coil_get,
 *     coil_timing and coil_adjoint synchronise with the host.
 *   - A handle is not thread-safe: use one handle per host thread.
 */
#ifndef COIL_H
#define COIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum coil_status {
    COIL_OK = 0,
    COIL_E_INVAL = -1,     /* invalid argument or configuration */
    COIL_E_NOMEM = -2,     /* workspace too small, or a host allocation failed */
    COIL_E_HIP = -3,       /* a HIP runtime call failed; message in coil_last_error */
    COIL_E_NONFINITE = -4, /* a non-finite value or a non-positive pivot appeared */
    COIL_E_STATE = -5      /* call not valid in the handle's current state */
};

enum coil_precision {
    COIL_FP64 = 0,  /* everything in FP64 */
    COIL_MIXED = 1  /* field pass in FP32 pair arithmetic: kernel values far from
                       k -> 1 evaluated in FP32, those with k > near_k evaluated in
                       FP64 (from FP64 arguments) and rounded to FP32; FP32
                       products and partial sums, the partial sums of every 16W
                       sources (TRANSLATION) or 64 sources (DIRECT, with a Kahan
                       correction across them) added into FP64; FFT: the kernel
                       values' spectra stored in FP32, the DFTs and the
                       products' sums in FP64; all state (I, Phi, u, T, Q) in
                       FP64 */
};

/* Geometry of the heat step and of the element volumes (the field and the
   inductances always treat elements as coaxial rings).  PLANAR replaces the
   ring volumes 2 pi r d^2 and face areas 2 pi r d by d^2 and d (per metre of
   depth): a test geometry for the heat step against planar closed forms. */
enum coil_geometry { COIL_AXISYMMETRIC = 0, COIL_PLANAR = 1 };

/* Inter-wire induction in each wire's circuit equation (paper, Methods,
   "Numerical Algorithm": a wire is first driven by the field of the transport
   current of the other wires; later iterations update it from the net currents
   of all subelements).  TRANSPORT: the other wires enter through the flux of
   their transport current only (the first iteration, which the paper finds
   sufficient for large coils).  FULL: the flux of every element current of the
   coil enters, solved to convergence each step (cg_tol, cg_max_iter). */
enum coil_coupling { COIL_COUPLE_TRANSPORT = 0, COIL_COUPLE_FULL = 1 };
/* FULL solves, per step, A dI + dt P U = b with P^T dI = dI_t 1 (A the coil's
   inductance matrix plus dt diag(2 pi r E'/d^2), P the element-to-wire
   incidence) by conjugate gradients on the zero-net-current corrections of the
   transport-only solution, preconditioned by the per-wire constrained solves,
   with an FP64 all-pairs flux pass as the product (in either precision).
   Eager stepping synchronises with the host every 8 iterations to stop at
   convergence; a captured graph holds all cg_max_iter iterations, those after
   convergence returning at once.  The adjoint is not available for it. */

/* Subelement model (paper, Results, the numerical-algorithm paragraph and the
   one before it: a wire's subelements, separated by resistive barriers, are
   uncoupled under an external field, each with zero net current, and coupled
   under transport current; J = J_H + J_I, both computed from the resistivity of
   the total J^k).  With subelements = s >= 1 the element current is I_H + I_I:
   per wire and step, A dI_H = b_H - P (dt U_s) with P^T dI_H = 0 (one loop
   voltage per subelement, P the element-to-subelement incidence) and
   A dI_I = b_I - dt U_I 1 with 1^T dI_I = dI_t, A = M_ww + dt diag(2 pi r E'/d^2),
   b_H = -dI_t Psi_u - pi r^2 dB_a - dt 2 pi r rho J_H, b_I = -dt 2 pi r rho J_I,
   rho = E/J of the total J^k (E' where J = 0).  s = 1 gives the wire model's
   currents.  COIL_F_UW is the element mean of the loop voltages,
   U_I + mean_s U_s.  Setting COIL_F_I leaves I_H as it is.  Transport-only
   coupling; no adjoint. */

/* Variable-step integration of the wire currents (paper, Methods, Numerical
   Algorithm, last sentence: Runge-Kutta with a variable time step for the
   electromagnetic equations, against divergences of the stiff power law).
   With em_tol > 0 each wire integrates its currents over the step with B^k and
   T^k (so Jc) held, in substeps h = dt / 2^m of the linearised implicit Euler
   step: an attempt takes one step of h and two of h/2 (the local law
   re-evaluated at the midpoint); err = max_e |I2 - I1| / (em_tol max(|I2|,
   Jc d^2)); err <= 1 keeps the extrapolated 2 I2 - I1 (second order,
   L-stable), otherwise m grows by one (the finest level is kept whatever err);
   after a kept substep with err <= 1/4 at a multiple of 2h, m falls by one.
   Every step starts at m = 0.  q and U_w are the substeps' averages (the half
   steps' E_lin J^{new}; 2 U2 - U1).  A wire whose resistive diagonal is below
   FP64 resolution takes its exact one-substep linear step.  Transport-only
   coupling, wire model; no adjoint. */

/* Heat step (paper, Methods, heat paragraph).  EXPLICIT: sub-cycled explicit
   finite volumes (heat_substeps).  ADI: alternating-direction implicit, one
   radial and one axial tridiagonal sweep per step. */
enum coil_heat { COIL_HEAT_EXPLICIT = 0, COIL_HEAT_ADI = 1 };
/* ADI (Peaceman-Rachford): per step, with the coefficients at T^n and q held,
   a half step implicit along r (one tridiagonal system per grid column) and
   one implicit along z (per grid row); the enthalpy takes the two half steps'
   inflow, so the energy balance is exact.  Face conductances
   A / (d/(2 k_e) + d/(2 k_f) + R_ins), border A / (1/h + d/(2 k_e)).
   Unconditionally stable, not monotone for steps far beyond the explicit
   limit.  Coils of at most 1536 elements per grid side; no adjoint. */

/* Field-pass evaluation.  Both compute the same all-pairs sum (every pair
   contributes G_B(e,j) I_j once):
   DIRECT evaluates K, E per pair on the fly (tiled N-body sum, any element
   positions);
   TRANSLATION uses that on a coil's regular (r,z) grid G_B depends on
   (i_r, j_r, i_z - j_z) only: per tile each distinct kernel value is evaluated
   once and reused along z (a per-row-pair 1-D convolution); in mixed
   precision the values with k > near_k come from a table evaluated once at
   coil_init, all others are evaluated on the fly every pass.  AUTO =
   TRANSLATION.
   FFT uses the same invariance the other way round: each row-pair
   convolution, zero-padded to a power of two L >= 2 n_z - 1, is a product of
   DFTs.  coil_init evaluates every kernel value once in FP64, transforms it
   (FP64) and keeps per coil two real n_r x n_r matrices per bin (L/2 + 1
   bins: G^_z is real as g_z is even in z, G^_r imaginary as g_r is odd),
   FP32 in COIL_MIXED, FP64 in COIL_FP64: 2 (L/2+1) n_r^2 reals, about
   4 n_r^2 n_z for n_z a power of two (1.9 GB for 480 x 800 in FP32); in
   COIL_FP64 a coil of n_r <= 256 keeps G^_r's matrix, symmetric in the two
   rows, as its packed upper triangle (about 1.5 (L/2+1) n_r^2 reals).  A
   pass transforms the source rows (FP64 DFTs), streams the matrices once
   (FP64 sums) and transforms the target rows back.  coil_run then also puts
   each step's heat step and reductions on a second stream of its own
   (created at coil_init, default priority), overlapping the next field
   pass, and joins it before returning.  Only selectable at coil_init (the autotuner then also
   times it).  With COIL_COUPLE_FULL the coupled solve's flux passes use the
   same scheme with the mutual-inductance kernel's spectra (one real matrix
   per bin, FP64: (L/2 + 1) n_r^2 more reals); otherwise they are
   TRANSLATION passes. */
enum coil_algo { COIL_ALGO_AUTO = 0, COIL_ALGO_DIRECT = 1, COIL_ALGO_TRANSLATION = 2, COIL_ALGO_FFT = 3 };

/* fields for coil_get / coil_set_state */
enum coil_field {
    COIL_F_I = 0,     /* element current, A                (settable) */
    COIL_F_J = 1,     /* current density I/d^2, A/m^2 */
    COIL_F_BR = 2,    /* field at the element centre, T (from the last field pass) */
    COIL_F_BZ = 3,
    COIL_F_T = 4,     /* temperature, K                    (settable) */
    COIL_F_PHI = 5,   /* accumulated flux linkage, Wb */
    COIL_F_QW = 6,    /* per-wire time-integrated Joule heat, J   (N_w entries) */
    COIL_F_UW = 7,    /* per-wire loop voltage of the last step, V (N_w entries) */
    COIL_F_E = 8,     /* electric field of the last step, V/m */
    COIL_F_EP = 9,    /* dE/dJ of the last step */
    COIL_F_U = 10,    /* enthalpy per volume relative to the bath, J/m^3 */
    COIL_F_Q = 11,    /* Joule source of the last step, W/m^3 */
    COIL_F_PSI = 12,  /* transport-flux pattern, Wb/A */
    COIL_F_R = 13,    /* element radius, m */
    COIL_F_Z = 14,    /* element height, m */
    COIL_F_DI = 15,   /* current increment of the last step, A */
    COIL_F_JC = 16,   /* critical current density of the last step, A/m^2 */
    /* per-wire flux-jump and quench diagnostics (N_w entries each; paper,
       Results: the criterion |J/Jc| > 1 for the nucleation of a flux jump in a
       wire, and rho > 0.95 rho_n for its quench, Fig. 4 and Fig. 6), from the
       local law of each step k (J^k, B^k, T^k): */
    COIL_F_ONSET = 17,    /* first step k with max over the wire |J|/Jc > 1 (Jc <= 0 with
                             J != 0 counts), -1 if none yet */
    COIL_F_QUENCH = 18,   /* first step k with rho_w = sum V E J / sum V J^2 > 0.95 rho_n
                             (rho_n > 0 only), -1 if none yet */
    COIL_F_Q_ONSET = 19,  /* the wire's Joule heat accumulated before its onset step, J */
    COIL_F_Q_QUENCH = 20, /* ... before its quench step, J */
    COIL_F_T_QUENCH = 21, /* the wire's largest T^k at its quench step, K */
    COIL_F_P_QUENCH = 22, /* its power density sum V E J / sum V at the quench step, W/m^3 */
    COIL_F_IH = 23,       /* subelement model: the field-driven component I_H of the element
                             current, A (I - I_H is the transport component) */
    COIL_F_EM_SUBSTEPS = 24  /* variable step: substeps each wire took in the last step (N_w) */
};

typedef struct {
    /* geometry and drive, one entry per coil (host arrays, copied at init) */
    int32_t n_coils;
    const int32_t *layers, *turns, *ne;   /* wires radial, axial; elements per wire side */
    const double *r_inner, *z_center, *wire_side; /* m */
    const double *ramp;                   /* transport current ramp, A/s (I_t = I0 + ramp t) */
    double dBa_dt;                        /* background axial field ramp, T/s */
    /* E-J law and Jc(B, T, eps) */
    double Ec, n, Jc0, Tc, B0, eps_coef, eps_pow;
    /* heat: C = C0 (T/T_ref)^cp_exp, constant k0 and h0, bath T_bath */
    double C0, T_ref, cp_exp, k0, h0, T_bath;
    double dt;              /* s */
    int32_t heat_substeps;  /* 0 = automatic: max(1, ceil(dt / (0.9 h_max))) */
    int32_t precision;      /* enum coil_precision */
    double near_k;          /* mixed mode: pairs with k > near_k run in FP64 (0 -> 0.99) */
    int32_t tile_targets;   /* field-pass tile: targets per workgroup (0 -> 256) */
    int32_t tile_sources;   /* sources per work item (0 -> automatic) */
    int32_t grid_limit;     /* 0: DIRECT: one workgroup per work item; TRANSLATION: one
                               workgroup per slot the GPU holds at once, each taking the
                               next work item in list order when free; > 0: persistent
                               grid of at most this many workgroups striding over the
                               work items (both evaluations) */
    int32_t algo;           /* enum coil_algo: how the field pass is evaluated */
    /* ---- options of the extended model; zero / NULL everywhere is the model of the
       benchmark configurations ---- */
    const double *I0;       /* per coil: transport current at t = 0, A, carried evenly by
                               the elements of each wire (NULL = 0); I_t = I0 + ramp t */
    double rho_n;           /* normal-state resistivity, Ohm m, in parallel with the power
                               law: rho = rho_pl rho_n / (rho_pl + rho_n), rho_pl = E/J of
                               the power law; Jc <= 0 is then the normal state E = rho_n J.
                               0 = pure power law (Jc <= 0 with J != 0 is an error) */
    double k_exp, h_exp;    /* k = k0 (T/T_ref)^k_exp, h = h0 (T/T_ref)^h_exp (paper: both
                               proportional to T^3); non-zero needs heat_solver = ADI */
    double ins_R0;          /* insulation between wires (composite cross-section): thermal
                               resistance per area, m^2 K / W, of every face between two
                               wires, scaled by (T_ref / T_face)^k_exp; needs ADI (0 = none) */
    int32_t geometry;       /* enum coil_geometry */
    int32_t coupling;       /* enum coil_coupling */
    int32_t heat_solver;    /* enum coil_heat */
    int32_t cg_max_iter;    /* COIL_COUPLE_FULL: iterations per step at most (0 -> 100) */
    double cg_tol;          /* COIL_COUPLE_FULL: relative residual to reach (0 -> 1e-12) */
    int32_t subelements;    /* subelement model: s x s square subelements of ne/s x ne/s
                               elements per wire (1 <= s <= 4, ne a multiple of s for every
                               coil; 0 = one current per element, the wire model) */
    double em_tol;          /* > 0: variable-step integration of the wire currents within a
                               step with this relative tolerance; 0 = one step of dt */
    int32_t em_max_level;   /* variable step: finest substep dt / 2^em_max_level (0 -> 10;
                               at most 16) */
} coil_config;

typedef struct {
    /* host arrays in public order, copied at init; NULL means all ones (jc0_mult,
       c_wire) or all zeros (strain) */
    const double *jc0_mult;  /* N: per-element Jc0 multiplier mu_e */
    const double *strain;    /* N: per-element strain eps_e */
    const double *c_wire;    /* N_w: per-wire Jc multiplier c_w */
    const double *k_mult;    /* N: thermal conductivity multiplier of each element (the
                                composite map; NULL = all ones; not all ones needs ADI) */
} coil_inputs;

typedef struct {
    size_t workspace_bytes;  /* device bytes coil_init needs */
    int64_t n_elem, n_wire;
    int32_t heat_substeps;   /* the substep count the run will use */
    int32_t n_work_items;    /* field-pass work items */
} coil_sizes;

typedef struct coil_s coil_t;

/* diag[] passed to a report callback: 0 t, 1 step, 2 I_t of coil 0, 3 max|B|,
   4 T_peak, 5 Q, 6 sum_w U_w, 7 max |J|/Jc of the last step */
typedef void (*coil_report_fn)(const double *diag, int32_t ndiag, void *user);

/* Sizes for a configuration.  No device work. */
int coil_query(const coil_config *cfg, coil_sizes *out);

/* Build a handle for the paper's model coil (Methods, Numerical Algorithm and
   Fig. 2(a): N_x x N_y wires of an axisymmetric solenoid, each split into
   current elements): validate, carve `workspace` (device memory, >= workspace_bytes,
   256-byte aligned), precompute geometry, per-layer inductance blocks (host,
   FP64), the transport-flux pattern (device, FP64 all-pairs pass), in mixed
   precision the near kernel values of the translation pass (device, FP64,
   stored in FP32), heat conductances, and zero the state (I = 0, T = T_bath,
   Phi = 0, Q = 0).  COIL_E_INVAL also when the near-value table would exceed
   2^31 entries.
   `stream` is a hipStream_t (NULL = default stream).  Synchronises once. */
int coil_init(const coil_config *cfg, const coil_inputs *in, void *workspace,
              size_t workspace_bytes, void *stream, coil_t **out);

/* Enqueue one time step k -> k+1 in the order of the paper's key subroutine
   (Methods, Numerical Algorithm and the Fig. 2(b) flow chart; the heat
   paragraph): field pass, local law + wire solve, heat step, reductions.
   Asynchronous. */
int coil_step(coil_t *h);

/* nsteps steps of coil_step (the paper's time loop under a ramped transport
   current and background field).  If report_every > 0 and cb != NULL, synchronise every
   report_every steps and call cb; returns COIL_E_NONFINITE if the status word
   shows a non-finite value at a report point or at the end (state left as is). */
int coil_run(coil_t *h, int64_t nsteps, int64_t report_every, coil_report_fn cb, void *user);

/* Only the field pass (step 1: the field at every element from the currents
   of all elements plus the background, paper, Methods, Numerical Algorithm)
   on the current currents and time; results in COIL_F_BR / COIL_F_BZ.
   Asynchronous. */
int coil_compute_field(coil_t *h);

/* Copy a field of the state (current, field, temperature, flux, the per-wire
   flux-jump and quench records of the paper's Results) out in public order.
   dst is device memory if dst_on_device,
   else host memory (then the call synchronises).  count must be >= the
   field's length (N, or N_w for per-wire fields). */
int coil_get(coil_t *h, int32_t field, double *dst, int64_t count, int32_t dst_on_device);

/* Overwrite a settable field (COIL_F_I, COIL_F_T) from public order; setting T
   also sets the enthalpy u = u(T).  Test and resume hook. */
int coil_set_state(coil_t *h, int32_t field, const double *src, int64_t count,
                   int32_t src_on_device);

/* Synchronise and read scalars: 0 t, 1 step, 2 Q, 3 T_peak, 4 sum U_w,
   5 max |J|/Jc, 6 heat out through the borders, 7 stored heat sum V u,
   8 status flags, 9 T_peak element (public index, -1 if none), 10 T_peak step,
   11 heat substeps, 12 field-pass work items, 13 conjugate-gradient iterations
   of the last step's coupled solve and 14 its final relative residual
   sqrt(r^T S r / r_0^T S r_0) (both 0 without COIL_COUPLE_FULL).  Writes
   min(n, 15) values. */
int coil_scalars(coil_t *h, double *dst, int32_t n);

/* Back to the t = 0 state (keeps the precompute). */
int coil_reset(coil_t *h);

/* Field at npts arbitrary points (host arrays, metres; r >= 0) from the current
   element currents of every coil, FP64 direct sum of the coaxial-ring field
   (the field the paper maps over the coil, Results, Figs. 3 and 5); B_r = 0 on the axis.  The
   background field is not included.  Synchronises. */
int coil_field_at(coil_t *h, int64_t npts, const double *r, const double *z, double *Br, double *Bz);

/* ---- allocation-free probes ----
   For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the field of
   coil_field_at (B_r, B_z in T at npts points (r, z) in metres, r >= 0, from
   the current element currents of every coil, FP64 direct sum, background
   field excluded, B_r = 0 on the axis), with r, z, Br and Bz DEVICE arrays of
   npts doubles.  Asynchronous on the handle's stream; calls no hipMalloc,
   hipFree or allocating library routine.  The sources are split into chunks
   whose partial sums live in one static device array of
   COIL_FIELD_AT_SCRATCH_BYTES per GPU (held until the process ends), shared by
   every handle and call on that GPU: calls that overlap on one GPU race.  Its
   address is taken once per device at coil_init.  COIL_E_INVAL when npts
   exceeds COIL_FIELD_AT_SCRATCH_BYTES / 16 (524,288 points).  Results agree
   with coil_field_at to rounding (the chunks are summed in a fixed order). */
#define COIL_FIELD_AT_SCRATCH_BYTES (8u << 20)
int coil_field_at_noalloc(coil_t *h, int64_t npts, const double *r, const double *z, double *Br, double *Bz);

/* Host snapshot of the state (I, u, T, Phi, Q_w, the per-wire onset and quench
   diagnostics, step, Q, T_peak and its argmax, heat outflow, status) for
   checkpoint and resume.  coil_save with
   host_buf = NULL only reports the size in *needed.  coil_load restores a
   snapshot taken from a handle of the same configuration; stepping on from it
   reproduces the uninterrupted run bitwise.  Both synchronise. */
int coil_save(coil_t *h, void *host_buf, size_t bytes, size_t *needed);
int coil_load(coil_t *h, const void *host_buf, size_t bytes);

/* Kernel timing with HIP events on the handle's stream.  enable = 1 starts
   recording every phase, 2 only phase 0 (two events per step instead of
   eight, for timing runs that should stay close to untimed ones); either
   clears the totals.  0 stops; other values give COIL_E_INVAL.
   coil_timing_read synchronises and returns per-phase totals: ms[p] and
   launches[p] for p = 0 field pass (the all-pairs kernel alone; the
   translation evaluation's reordering of the currents runs before it),
   1 local law + wire solve, 2 heat substeps, 3 reductions (n >= 4). */
int coil_timing(coil_t *h, int32_t enable);
int coil_timing_read(coil_t *h, double *ms, int64_t *launches, int32_t n);

/* Capture `steps` consecutive coil_step calls into a HIP graph; subsequent
   coil_run calls replay it in chunks of `steps` (remainder eagerly).  steps = 0
   drops the graph.  The graph holds only kernel nodes. */
int coil_graph(coil_t *h, int64_t steps);

/* Replace the per-wire Jc multipliers c_w (N_w host values, or NULL to keep)
   and the per-coil ramp rates (n_coils host values, or NULL to keep); the state
   is not touched.  Synchronises. */
int coil_set_params(coil_t *h, const double *c_wire, const double *ramp);

/* ---- discrete adjoint (checkpointed) ----
   Objective J = wQ Q + wTpeak T_peak after nsteps from t = 0, with Q the
   time-integrated Joule heat and T_peak the peak temperature (paper, Results:
   per-wire time-integrated Joule heat as the quantity that orders flux-jump and
   quench propagation).  coil_adjoint resets the handle, runs the forward pass
   storing the state (I, u, T) every ckpt_every steps (and, if store_field, the
   field B of every step), then the reverse sweep: each segment is recomputed
   from its checkpoint with the step's intermediates recorded, and the adjoint
   of every step is applied in reverse order (heat substeps, Joule source,
   per-wire KKT system with the same Cholesky factor, local law and Jc, and a
   transposed all-pairs field pass).  The peak temperature's gradient is that
   of its element and step (ties resolved to the lowest step, then the lowest
   public element index); zero-measure kinks (|B| = 0, T = Tc, J = 0) take the
   zero branch.
   Outputs: g_c_wire[N_w] = dJ/dc_w, g_ramp[n_coils] = dJ/d(ramp rate),
   objectives[2] = (Q, T_peak).  `workspace` is caller-owned device memory of
   at least coil_adjoint_query() bytes (256-byte aligned); it is free again on
   return.  The handle is left reset to t = 0.  Synchronises.
   Returns COIL_E_NONFINITE if the forward pass produced a non-finite value,
   COIL_E_INVAL for a handle with coupling COIL_COUPLE_FULL. */
int coil_adjoint_query(coil_t *h, int64_t nsteps, int32_t ckpt_every, int32_t store_field,
                       size_t *bytes);
int coil_adjoint(coil_t *h, int64_t nsteps, double wQ, double wTpeak, int32_t ckpt_every,
                 int32_t store_field, void *workspace, size_t bytes, double *g_c_wire,
                 double *g_ramp, double *objectives);

/* Test hook: out = G^T bbar, the transposed field pass.  bbar_r, bbar_z, out
   in public order (host, or device if on_device).  out_j = sum_e dB_e/dI_j .
   bbar_e over the elements e of j's coil.  Overwrites the stored field
   (COIL_F_BR/BZ) and COIL_F_DI.  Synchronises. */
int coil_field_transpose(coil_t *h, const double *bbar_r, const double *bbar_z, double *out,
                         int32_t on_device);

/* ---- field-pass tiling (batched and single coils) ----
   coil_set_tiles: switch to the DIRECT evaluation with tile_targets in
   {64, 128, 256} targets per workgroup, chunks = source chunks per coil (0 =
   automatic, at most 16) and grid_limit = 0 for one workgroup per work item or
   > 0 for a persistent grid striding over the (coil, target block, source
   chunk) items.  Drops a captured graph.
   coil_autotune: times the candidates over `reps` field passes on the
   handle's current currents and keeps the fastest: TRANSLATION with 4, 8, 16, 32
   or 64 source-row groups per target row segment (launched as a work queue,
   grid_limit 0), and DIRECT with 3 tile sizes x
   5 chunk counts x 3 grid shapes.  A candidate whose first (timed) pass is
   over 3x the best so far is not timed further, nor is the rest of a family
   whose first three candidates all were.  With cache_path it first looks the
   configuration up in that JSON-lines file (key: arch / precision / log2 pairs /
   coils) and appends a new choice.  chosen[4] (optional) receives (algo, p1,
   p2, p3): (2, groups, 0, 0) or (1, tile_targets, chunks, grid_limit).
   Results differ between candidates only by summation order. */
int coil_set_tiles(coil_t *h, int32_t tile_targets, int32_t chunks, int32_t grid_limit);
int coil_autotune(coil_t *h, int32_t reps, const char *cache_path, int32_t *chosen);

/* Segment width of the TRANSLATION evaluation: w = 0 lets the planner cut each
   coil's rows into the widths of least estimated time (per-width throughput
   measured on this GPU); w in [2, 8] uses segments of 64 w targets (w per
   thread) everywhere.  Applies to the forward and the transposed pass, whether
   or not TRANSLATION is the current evaluation; keeps the source-row split.
   Results differ between widths only by summation order.  Drops a captured
   graph.  COIL_E_INVAL for other w, COIL_E_STATE during capture. */
int coil_set_widths(coil_t *h, int32_t w);

/* Work of one field pass as planned: out[0] ordered (target, source) pairs,
   out[1] Green's-function evaluations the pass performs (= pairs for DIRECT;
   TRANSLATION in mixed mode leaves out the near values made at set-up),
   out[2] the algorithm (enum coil_algo), out[3] work items, out[4] direct-pass
   targets per workgroup, out[5] workgroups of the launch.  Writes min(n, 6)
   values.  No device work. */
int coil_field_stats(coil_t *h, double *out, int32_t n);

void coil_destroy(coil_t *h);  /* does not free the caller's workspace */
const char *coil_last_error(void);

/* ---- test hook: library elliptic integrals evaluated on the host ----
   precision COIL_FP64 or COIL_MIXED (FP32 polynomial); no device work. */
int coil_host_ellip(double m1, int32_t precision, double *K, double *E);

#ifdef __cplusplus
}
#endif
#endif /* COIL_H */
