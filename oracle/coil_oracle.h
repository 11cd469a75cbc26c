/*
 * coil_oracle.h -- plain, slow FP64 CPU oracle of the coil quench hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this library.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * What it computes (paper: Methods, "Numerical Algorithm" and the heat
 * paragraph that follows the figures; Fig. 2(b) flow chart):
 *   - each current element is a coaxial ring (axisymmetric cross-section);
 *   - per time step: the all-pairs ring field B from every element current,
 *     the local power law E-J with Jc(B,T,eps), a per-wire A-V solve that
 *     enforces the wire's transport current, then the explicit heat step
 *     c dT/dt = div(k grad T) + E.J with a Robin condition on the four
 *     borders of the cross-section.
 * Readings where the paper is silent are listed at the top of coil_oracle.c.
 *
 * Element order ("public order"): coils concatenated, inside a coil the
 * (r,z) grid row-major, e = i_r * n_z + i_z.  Wire order w = layer*turns+turn.
 */
#ifndef COIL_ORACLE_H
#define COIL_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXC 64

typedef struct {
    int n_coils;
    int layers[ORC_MAXC], turns[ORC_MAXC], ne[ORC_MAXC];
    double r_inner[ORC_MAXC], z_center[ORC_MAXC], wire_side[ORC_MAXC];
    double ramp[ORC_MAXC], I0[ORC_MAXC];
    double dBa_dt;
    double Ec, n, Jc0, Tc, B0, eps_coef, eps_pow;
    double C0, T_ref, cp_exp, k0, h0, T_bath;
    double dt;
    int n_sub;   /* heat substeps per step; 0 = automatic stability rule */
    int planar;  /* 1: heat in planar (Cartesian) geometry, test use only */
    double rho_n;  /* normal-state resistivity in parallel with the power law (0 = off) */
    int coupling;  /* 0: other wires through their transport current (R3);
                      1: every element current of the coil (dense solve; coils of
                      at most 4096 elements) */
    int heat_solver;  /* 0: explicit, sub-cycled; 1: alternating-direction implicit */
    double k_exp, h_exp;  /* ADI: k = k0 (T/T_ref)^k_exp k_mult_e, h = h0 (T/T_ref)^h_exp */
    double ins_R0;    /* ADI: thermal resistance per area of the insulation between
                         wires, m^2 K / W, scaled by (T_ref / T_face)^k_exp (0 = none) */
    int subelements;  /* 0: one current per element (the wire model); s >= 1: the
                         two-component subelement model with s x s square
                         subelements of ne/s x ne/s elements per wire */
    double em_tol;    /* > 0: variable-step integration of each wire's currents within
                         the step (substeps dt / 2^m, step-doubling error control with
                         this relative tolerance); 0: one step of dt */
    int em_max_level; /* finest substep dt / 2^em_max_level (0 -> 10) */
} orc_cfg;

typedef struct orc_sim orc_sim;

/* ---- pure functions (pinned by the unit tests) ---- */
/* complete elliptic integrals K(m), E(m) with the complementary parameter
   m1 = 1 - m passed directly (Carlson symmetric forms). */
void   orc_ellip(double m1, double *K, double *E);
double orc_carlson_rf(double x, double y, double z);
double orc_carlson_rd(double x, double y, double z);
/* field at (r,z) of a coaxial filament ring of radius a at height zs, current I */
void   orc_ring_B(double a, double zs, double r, double z, double I, double *Br, double *Bz);
/* mutual inductance of two coaxial filament rings (Maxwell) */
double orc_ring_M(double a, double zs, double r, double z);
/* self inductance of a ring of radius r with a square d x d section */
double orc_self_L(double r, double d);

/* OpenMP threads the oracle's parallel loops use */
int    orc_threads(void);

/* ---- simulation ---- */
/* inputs in public order: jc0_mult[N], strain[N], c_wire[Nw].  Returns NULL
   on invalid configuration. */
orc_sim *orc_create(const orc_cfg *cfg, const double *jc0_mult, const double *strain,
                    const double *c_wire);
/* field_only = 1: geometry only (no inductance blocks, no transport-flux
   pattern); orc_field_targets/points work, orc_step returns -1 */
orc_sim *orc_create_ex(const orc_cfg *cfg, const double *jc0_mult, const double *strain,
                       const double *c_wire, int field_only);
void   orc_destroy(orc_sim *s);
long   orc_n_elem(const orc_sim *s);
long   orc_n_wire(const orc_sim *s);
int    orc_n_sub(const orc_sim *s);
/* one time step; returns 0, or -4 when a non-finite value appeared */
int    orc_step(orc_sim *s);
int    orc_run(orc_sim *s, long nsteps);

/* field names for orc_get / orc_set */
enum { ORC_I = 0, ORC_J = 1, ORC_BR = 2, ORC_BZ = 3, ORC_T = 4, ORC_PHI = 5,
       ORC_QW = 6, ORC_UW = 7, ORC_E = 8, ORC_EP = 9, ORC_U = 10, ORC_Q = 11,
       ORC_PSI = 12, ORC_R = 13, ORC_Z = 14, ORC_V = 15, ORC_JC = 16, ORC_DI = 17,
       /* per-wire flux-jump and quench diagnostics (N_w entries each):
          ORC_ONSET  first step k with max_e |J_e^k| / Jc_e^k > 1, -1 if none;
          ORC_QUENCH first step k with rho_w^k > 0.95 rho_n, -1 if none, where
                     rho_w^k = sum_e V E J / sum_e V J^2 of the step's local law;
          ORC_Q_ONSET, ORC_Q_QUENCH  the wire's Joule heat accumulated before
                     those steps; ORC_T_QUENCH the wire's max T^k and
                     ORC_P_QUENCH its power density sum V E J / sum V at the
                     quench step */
       ORC_ONSET = 18, ORC_QUENCH = 19, ORC_Q_ONSET = 20, ORC_Q_QUENCH = 21,
       ORC_T_QUENCH = 22, ORC_P_QUENCH = 23,
       /* per-element conductivity multiplier of the ADI heat step (settable,
          default 1): the composite map */
       ORC_KMULT = 24,
       /* the field-driven component I_H of the element current (subelement
          model; I - I_H is the transport component) */
       ORC_IH = 25,
       /* per wire: substeps of the last step (variable-step EM integration) */
       ORC_EMSUB = 26 };
int    orc_get(const orc_sim *s, int field, double *dst, long count);
int    orc_set(orc_sim *s, int field, const double *src, long count);
/* scalars: [0]=t, [1]=step, [2]=Q, [3]=T_peak, [4]=sum U_w, [5]=max |J|/Jc,
   [6]=heat out through the borders, [7]=stored heat sum V u, [8]=I_t,
   [9]=argmax element of T_peak, [10]=argmax step of T_peak, [11]=n_sub */
int    orc_scalars(const orc_sim *s, double *dst, int n);

/* field sum B = sum_j G_B(e,j) I_j at the listed target elements, for an
   arbitrary current vector I[N] (public order); background field excluded. */
void   orc_field_targets(const orc_sim *s, const double *I, long nt, const long *tgt,
                         double *Br, double *Bz);
/* the same sum at arbitrary points (r,z) of coil `coil` */
void   orc_field_points(const orc_sim *s, const double *I, long np, const double *r,
                        const double *z, double *Br, double *Bz);
/* elements of wire w (public indices), returns count */
int    orc_wire_elems(const orc_sim *s, long w, long *dst);

/* tangent-linear (forward-mode) derivative (coupling 0, the explicit heat
   step and the wire model, subelements 0, only; returns -1 otherwise) of the
   run's objectives
   Q (time-integrated Joule heat) and T_peak along the direction
   (dc_wire[Nw], dramp[n_coils]) for nsteps from the initial state.
   obj[2] = (Q, T_peak), dobj[2] = directional derivatives. */
int    orc_tangent(const orc_cfg *cfg, const double *jc0_mult, const double *strain,
                   const double *c_wire, const double *dc_wire, const double *dramp,
                   long nsteps, double *obj, double *dobj);

#ifdef __cplusplus
}
#endif
#endif
