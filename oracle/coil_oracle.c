/*
 * coil_oracle.c -- plain, slow, FP64 CPU oracle of the coil quench hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.
 *
 * Method (paper, Methods: "Numerical Algorithm", the heat-diffusion paragraph,
 * the E-J paragraph; Fig. 1(b), Fig. 2(a,b)):
 *   The solenoid is rotationally symmetric, so its (r,z) cross-section is
 *   modelled.  Wires sit on a square array; each wire is split into square
 *   current elements, each element a coaxial ring carrying current I_e.
 *   Per time step k -> k+1:
 *     1. field: B_e = B_a(t_k) z + sum_{j != e} G_B(e,j) I_j (coaxial-ring
 *        Green's function with complete elliptic integrals);
 *     2. local law: Jc(B,T,eps), E = Ec (|J|/Jc)^n sgn J and dE/dJ, evaluated
 *        at step k (the paper evaluates the resistivity from J^k);
 *     3. per wire A-V solve: one loop voltage per wire enforces the transport
 *        current; the other wires drive the wire through the flux of their
 *        transport current (first iteration of the paper's scheme);
 *     4. heat: c dT/dt = div(k grad T) + E.J, Robin h (T - T0) on the four
 *        borders, explicit finite volumes on the enthalpy, sub-cycled;
 *     5. accumulate Joule heat Q, per-wire Q_w, peak temperature.
 *
 * Readings where the paper is silent (its constitutive laws, A-V details and
 * GPU algorithm are in the Supplementary Information, which is not available):
 *   R1 geometry: contiguous square wires, ne x ne square elements per wire.
 *   R2 self terms: the B self term of an element at its own centre is 0;
 *      ring self inductance mu0 r (ln(8r/g) - 2) with g the geometric mean
 *      distance of a square section, g = 0.4470491559036625 d.
 *   R3 inter-wire coupling in Faraday's law: transport current of the other
 *      wires only (static pattern Psi_u times dI_t); the all-pairs B from
 *      every element current enters through Jc(B).  Option coupling = 1: the
 *      flux of every element current of the coil (the converged form of the
 *      paper's field iteration), one dense constrained solve per coil.
 *   R4 A-V: 2 pi r_e E_e + U_w = -dPhi_e/dt, sum_{e in w} I_e = I_t.
 *   R5 time integrator: linearised backward Euler per wire.  Option em_tol > 0:
 *      variable-step integration of each wire within the step (substeps
 *      dt / 2^m with step-doubling error control; em_wire).
 *   Subelements (option subelements = s >= 1): a wire's ne x ne elements form
 *      s x s square subelements.  The element current is I_H + I_I: the
 *      field-driven part I_H keeps zero net current in every subelement
 *      (uncoupled subelements), the transport part I_I carries the wire's
 *      transport current (coupled); both respond through the same wire
 *      matrix, each driven by the resistivity rho^k = E/J of the total J^k
 *      times its own current (the paper's J_H and J_I).
 *   R6 order: field -> local -> wire solve -> heat; Jc, E from (B^k, T^k).
 *   R7 normal state: pure power law by default (Jc <= 0 with J != 0 is an
 *      error); with rho_n > 0 the power-law resistivity acts in parallel with
 *      the normal-state resistivity rho_n (flux creep, flux flow and normal
 *      state in one law), and Jc <= 0 is the normal state.
 *   R8 Joule source: q = (E + E' dI/d^2) J^{k+1}.
 *   R9 heat substeps n_sub = max(1, ceil(dt / (0.9 h_max))) (1e-9 relative
 *      tolerance on the quotient), h_max the explicit stability limit at T_bath.
 *   R10 axisymmetric finite volumes, half-cell series resistance at borders.
 *   R11 constant k and h, C = C0 (T/T_ref)^p, enthalpy form.  Option
 *      heat_solver = 1: the paper's ADI scheme with k and h proportional to
 *      (T/T_ref)^k_exp, (T/T_ref)^h_exp, a per-element conductivity map and an
 *      insulation resistance between wires (composite cross-section).
 * Every reading is listed with its justification in the design notes.
 *
 * Elliptic integrals: Carlson's symmetric forms R_F, R_D by the duplication
 * algorithm (B. C. Carlson, "Numerical computation of real or complex elliptic
 * integrals", Numer. Algorithms 10 (1995)).  Sums over sources use Neumaier's
 * compensated summation.  OpenMP parallelises over independent targets and
 * wires only; every sum is evaluated in a fixed order.
 */
#include "coil_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_MU0 (4.0e-7 * ORC_PI)
/* geometric mean distance of a unit square from itself:
   exp( integral over the square x square of ln|p - q| ) */
#define ORC_GMD_SQUARE 0.4470491559036625

/* ------------------------------------------------------------------ */
/* compensated summation                                               */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;
static void ns_add(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}
static double ns_val(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Carlson symmetric elliptic integrals                                */
/* ------------------------------------------------------------------ */
double orc_carlson_rf(double x, double y, double z) {
    const double r = 1.0e-16;
    const double x0 = x, y0 = y, z0 = z;
    const double A0 = (x + y + z) / 3.0;
    double A = A0;
    const double Q = pow(3.0 * r, -1.0 / 6.0) *
                     fmax(fabs(A0 - x0), fmax(fabs(A0 - y0), fabs(A0 - z0)));
    double p4 = 1.0;
    while (p4 * fabs(A) <= Q) {
        const double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        const double lam = sx * sy + sx * sz + sy * sz;
        A = 0.25 * (A + lam);
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
        p4 *= 4.0;
    }
    const double X = (A0 - x0) / (p4 * A);
    const double Y = (A0 - y0) / (p4 * A);
    const double Z = -(X + Y);
    const double E2 = X * Y - Z * Z;
    const double E3 = X * Y * Z;
    return (1.0 - E2 / 10.0 + E3 / 14.0 + E2 * E2 / 24.0 - 3.0 * E2 * E3 / 44.0) / sqrt(A);
}

double orc_carlson_rd(double x, double y, double z) {
    const double r = 1.0e-16;
    const double x0 = x, y0 = y, z0 = z;
    const double A0 = (x + y + 3.0 * z) / 5.0;
    double A = A0;
    const double Q = pow(0.25 * r, -1.0 / 6.0) *
                     fmax(fabs(A0 - x0), fmax(fabs(A0 - y0), fabs(A0 - z0)));
    double p4 = 1.0, sum = 0.0;
    while (p4 * fabs(A) <= Q) {
        const double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        const double lam = sx * sy + sx * sz + sy * sz;
        sum += 1.0 / (p4 * sz * (z + lam));
        A = 0.25 * (A + lam);
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
        p4 *= 4.0;
    }
    const double X = (A0 - x0) / (p4 * A);
    const double Y = (A0 - y0) / (p4 * A);
    const double Z = -(X + Y) / 3.0;
    const double XY = X * Y, Z2 = Z * Z;
    const double E2 = XY - 6.0 * Z2;
    const double E3 = (3.0 * XY - 8.0 * Z2) * Z;
    const double E4 = 3.0 * (XY - Z2) * Z2;
    const double E5 = XY * Z2 * Z;
    const double ser = 1.0 - 3.0 * E2 / 14.0 + E3 / 6.0 + 9.0 * E2 * E2 / 88.0
                     - 3.0 * E4 / 22.0 - 9.0 * E2 * E3 / 52.0 + 3.0 * E5 / 26.0;
    return ser / (p4 * A * sqrt(A)) + 3.0 * sum;
}

/* K(m) = R_F(0, 1-m, 1), E(m) = R_F(0, 1-m, 1) - (m/3) R_D(0, 1-m, 1) */
void orc_ellip(double m1, double *K, double *E) {
    if (m1 <= 0.0) { *K = INFINITY; *E = 1.0; return; }
    const double m = 1.0 - m1;
    const double rf = orc_carlson_rf(0.0, m1, 1.0);
    const double rd = orc_carlson_rd(0.0, m1, 1.0);
    *K = rf;
    *E = rf - (m / 3.0) * rd;
}

/* ------------------------------------------------------------------ */
/* ring Green's functions (coaxial filament loop; textbook closed forms) */
/* ------------------------------------------------------------------ */
void orc_ring_B(double a, double zs, double r, double z, double I, double *Br, double *Bz) {
    const double dz = z - zs;
    const double al2 = (r - a) * (r - a) + dz * dz;
    const double be2 = (r + a) * (r + a) + dz * dz;
    const double be = sqrt(be2);
    double K, E;
    orc_ellip(al2 / be2, &K, &E);
    const double pre = ORC_MU0 * I / (2.0 * ORC_PI * al2 * be);
    *Bz = pre * ((a * a - r * r - dz * dz) * E + al2 * K);
    *Br = (r > 0.0) ? pre * (dz / r) * ((a * a + r * r + dz * dz) * E - al2 * K) : 0.0;
}

double orc_ring_M(double a, double zs, double r, double z) {
    const double dz = z - zs;
    const double al2 = (r - a) * (r - a) + dz * dz;
    const double be2 = (r + a) * (r + a) + dz * dz;
    const double m1 = al2 / be2;
    double K, E;
    orc_ellip(m1, &K, &E);
    return ORC_MU0 * sqrt(be2) * (0.5 * (1.0 + m1) * K - E);
}

double orc_self_L(double r, double d) {
    return ORC_MU0 * r * (log(8.0 * r / (ORC_GMD_SQUARE * d)) - 2.0);
}

/* ------------------------------------------------------------------ */
/* local E-J law (paper, Methods, E-J paragraph; readings R7)          */
/* ------------------------------------------------------------------ */
/* E(J) and dE/dJ at one element for a given Jc.  Power law E = Ec x^n sgn J,
   x = |J| / Jc.  With rho_n > 0 the power-law resistivity
   rho_pl = E/J = (Ec/Jc) x^(n-1) is in parallel with rho_n:
   rho = rho_pl rho_n / (rho_pl + rho_n), E = rho J, so that
   dE/dJ = rho_n * p/(p + rho_n) * (n rho_n + p)/(rho_n + p) with p = rho_pl;
   Jc <= 0 (T >= Tc) is then the normal state E = rho_n J.  Returns 1 when the
   pure power law meets Jc <= 0 with J != 0 (no finite E). */
static int local_EJ(const orc_cfg *c, double J, double Jc, double *E, double *Ep, double *x) {
    if (c->rho_n > 0.0 && !(Jc > 0.0)) {
        *E = c->rho_n * J;
        *Ep = c->rho_n;
        *x = (J != 0.0) ? INFINITY : 0.0;
        return 0;
    }
    if (J == 0.0) { *E = 0.0; *Ep = 0.0; *x = 0.0; return 0; }
    if (!(Jc > 0.0)) { *E = NAN; *Ep = NAN; *x = INFINITY; return 1; }
    *x = fabs(J) / Jc;
    if (c->rho_n > 0.0) {
        const double p = c->Ec / Jc * pow(*x, c->n - 1.0);
        if (!isfinite(p)) { *E = c->rho_n * J; *Ep = c->rho_n; return 0; }
        const double sfr = p / (p + c->rho_n);
        *E = c->rho_n * sfr * J;
        *Ep = c->rho_n * sfr * ((c->n * c->rho_n + p) / (c->rho_n + p));
        return 0;
    }
    *E = c->Ec * pow(*x, c->n) * (J > 0.0 ? 1.0 : -1.0);
    *Ep = c->n * c->Ec / Jc * pow(*x, c->n - 1.0);
    return 0;
}

/* directional derivatives dE, dE' of the law above for perturbations dJ, dJc */
static void local_EJ_tangent(const orc_cfg *c, double J, double Jc, double dJ, double dJc,
                             double *dE, double *dEp) {
    *dE = 0.0;
    *dEp = 0.0;
    if (c->rho_n > 0.0 && !(Jc > 0.0)) { *dE = c->rho_n * dJ; return; }
    if (J == 0.0 || !(Jc > 0.0)) return;
    const double x = fabs(J) / Jc;
    if (c->rho_n > 0.0) {
        const double rn = c->rho_n, n = c->n;
        const double p = c->Ec / Jc * pow(x, n - 1.0);
        if (!isfinite(p)) { *dE = rn * dJ; return; }
        /* p = Ec |J|^(n-1) / Jc^n */
        const double dp = p * ((n - 1.0) * dJ / J - n * dJc / Jc);
        const double sfr = p / (p + rn), tfr = (n * rn + p) / (rn + p);
        const double dsfr = rn * dp / ((p + rn) * (p + rn));
        const double dtfr = (1.0 - n) * rn * dp / ((p + rn) * (p + rn));
        *dE = rn * (sfr * dJ + J * dsfr);
        *dEp = rn * (dsfr * tfr + sfr * dtfr);
        return;
    }
    const double sg = J > 0.0 ? 1.0 : -1.0;
    const double dx = x * (dJ / J - dJc / Jc);
    *dE = c->Ec * c->n * pow(x, c->n - 1.0) * dx * sg;
    *dEp = c->n * c->Ec * ((c->n - 1.0) * pow(x, c->n - 2.0) * dx / Jc - pow(x, c->n - 1.0) * dJc / (Jc * Jc));
}

/* ------------------------------------------------------------------ */
/* simulation state                                                    */
/* ------------------------------------------------------------------ */
struct orc_sim {
    orc_cfg cfg;
    long N, Nw;
    int n_sub;
    /* geometry, public order */
    double *r, *z, *d, *V;
    int *coil, *wire;
    long *coil_off, *wire_off;   /* first element of coil c; first slot of wire w in welem */
    long *welem;                 /* elements of each wire, local order a*ne + b */
    int  *wn;                    /* elements per wire */
    int  *wcoil;                 /* coil of wire */
    /* static material */
    double *jcs;                 /* Jc0 * mu_e * (1 - eps_coef |eps|^eps_pow) */
    double *cw;                  /* per-wire multiplier */
    /* precompute */
    double **Mww;                /* per wire, wn x wn row-major */
    double **Mc;                 /* coupling 1: per coil, its full N_c x N_c inductance matrix */
    double *psi;                 /* transport flux pattern per element */
    long *nb;                    /* 4 neighbours per element, -1 = border */
    double *G;                   /* 4 face conductances */
    double *Gb;                  /* border conductance (sum over border faces) */
    /* state */
    double *I, *u, *T, *Phi, *Br, *Bz, *E, *Ep, *Jc, *dI, *q, *Qw, *U;
    double Q, Tpeak, Qout, maxx, sumU;
    long step, Tpeak_e, Tpeak_k;
    /* per-wire flux-jump / quench diagnostics (see ORC_ONSET .. ORC_P_QUENCH) */
    double *onset, *quench, *Qon, *Qqu, *Tqu, *Pqu;
    double *kmult;               /* ADI heat: conductivity multiplier per element */
    double *IH;                  /* subelement model: field-driven component of I */
    double *emsub;               /* per wire: EM substeps of the last step */
    int field_only;  /* geometry only: no inductance blocks, no transport flux */
};

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

long orc_n_elem(const orc_sim *s) { return s->N; }
long orc_n_wire(const orc_sim *s) { return s->Nw; }
int  orc_n_sub(const orc_sim *s) { return s->n_sub; }

static double *dalloc(long n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static int cfg_valid(const orc_cfg *c) {
    if (c->n_coils < 1 || c->n_coils > ORC_MAXC) return 0;
    for (int i = 0; i < c->n_coils; ++i) {
        if (c->layers[i] < 1 || c->turns[i] < 1 || c->ne[i] < 1) return 0;
        if (!(c->wire_side[i] > 0) || !(c->r_inner[i] > 0)) return 0;
    }
    if (!(c->dt > 0) || !(c->Ec > 0) || !(c->n >= 1) || !(c->Jc0 > 0)) return 0;
    if (!(c->Tc > 0) || !(c->B0 > 0) || !(c->C0 > 0) || !(c->T_ref > 0)) return 0;
    if (!(c->k0 > 0) || !(c->h0 >= 0) || !(c->T_bath > 0)) return 0;
    if (!(c->rho_n >= 0) || !isfinite(c->rho_n)) return 0;
    if (c->coupling != 0 && c->coupling != 1) return 0;
    if (c->heat_solver != 0 && c->heat_solver != 1) return 0;
    if (!isfinite(c->k_exp) || !isfinite(c->h_exp) || !(c->ins_R0 >= 0) || !isfinite(c->ins_R0)) return 0;
    if (c->heat_solver == 0 && (c->k_exp != 0.0 || c->h_exp != 0.0 || c->ins_R0 != 0.0)) return 0;
    if (c->subelements < 0) return 0;
    for (int i = 0; i < c->n_coils && c->subelements >= 1; ++i)
        if (c->ne[i] % c->subelements != 0) return 0;
    if (c->subelements >= 1 && c->coupling != 0) return 0;
    if (!(c->em_tol >= 0.0) || !isfinite(c->em_tol) || c->em_max_level < 0 || c->em_max_level > 20) return 0;
    if (c->em_tol > 0.0 && (c->coupling != 0 || c->subelements != 0)) return 0;
    for (int i = 0; i < c->n_coils && c->coupling == 1; ++i)
        if ((long)c->layers[i] * c->turns[i] * c->ne[i] * c->ne[i] > 4096) return 0;
    for (int i = 0; i < c->n_coils; ++i)
        if (!isfinite(c->I0[i])) return 0;
    return 1;
}

/* enthalpy per volume relative to the bath and its inverse:
   u(T) = C0 T_ref/(p+1) [ (T/T_ref)^(p+1) - (T_bath/T_ref)^(p+1) ] */
static double u_of_T(const orc_cfg *c, double T) {
    const double p1 = c->cp_exp + 1.0;
    return c->C0 * c->T_ref / p1 * (pow(T / c->T_ref, p1) - pow(c->T_bath / c->T_ref, p1));
}
static double T_of_u(const orc_cfg *c, double u) {
    const double p1 = c->cp_exp + 1.0;
    const double x = p1 * u / (c->C0 * c->T_ref) + pow(c->T_bath / c->T_ref, p1);
    return c->T_ref * pow(x, 1.0 / p1);
}

/* heat conductances of element e (public index inside its coil grid) */
static void build_heat(orc_sim *s) {
    const orc_cfg *c = &s->cfg;
    for (int ci = 0; ci < c->n_coils; ++ci) {
        const int ne = c->ne[ci];
        const long nr = (long)c->layers[ci] * ne, nz = (long)c->turns[ci] * ne;
        const double d = c->wire_side[ci] / ne;
        const double rin = c->r_inner[ci];
        for (long ir = 0; ir < nr; ++ir)
            for (long iz = 0; iz < nz; ++iz) {
                const long e = s->coil_off[ci] + ir * nz + iz;
                const double re = s->r[e];
                /* faces: 0 = inner radial (ir-1), 1 = outer radial (ir+1),
                          2 = lower axial (iz-1), 3 = upper axial (iz+1) */
                const double rf_in = rin + (double)ir * d;
                const double rf_out = rin + (double)(ir + 1) * d;
                double area[4], gface[4];
                if (c->planar) {
                    area[0] = area[1] = area[2] = area[3] = d;
                } else {
                    area[0] = 2.0 * ORC_PI * rf_in * d;
                    area[1] = 2.0 * ORC_PI * rf_out * d;
                    area[2] = area[3] = 2.0 * ORC_PI * re * d;
                }
                long nbr[4];
                nbr[0] = (ir > 0) ? e - nz : -1;
                nbr[1] = (ir < nr - 1) ? e + nz : -1;
                nbr[2] = (iz > 0) ? e - 1 : -1;
                nbr[3] = (iz < nz - 1) ? e + 1 : -1;
                double gb = 0.0;
                for (int f = 0; f < 4; ++f) {
                    gface[f] = c->k0 * area[f] / d; /* centre-to-centre distance d */
                    s->nb[4 * e + f] = nbr[f];
                    if (nbr[f] >= 0) {
                        s->G[4 * e + f] = gface[f];
                    } else {
                        s->G[4 * e + f] = 0.0;
                        gb += (c->h0 > 0.0) ? area[f] / (1.0 / c->h0 + d / (2.0 * c->k0)) : 0.0;
                    }
                }
                s->Gb[e] = gb;
            }
    }
    /* explicit stability limit at the bath temperature */
    const double Cb = c->C0 * pow(c->T_bath / c->T_ref, c->cp_exp);
    double hmax = INFINITY;
    for (long e = 0; e < s->N; ++e) {
        double g = s->Gb[e];
        for (int f = 0; f < 4; ++f) g += s->G[4 * e + f];
        if (g > 0.0) {
            const double h = s->V[e] * Cb / g;
            if (h < hmax) hmax = h;
        }
    }
    if (c->heat_solver == 1) {
        s->n_sub = 1;  /* one implicit step */
    } else if (c->n_sub > 0) {
        s->n_sub = c->n_sub;
    } else {
        const double qt = c->dt / (0.9 * hmax);
        long ns = (long)ceil(qt * (1.0 - 1.0e-9));
        s->n_sub = (int)(ns < 1 ? 1 : ns);
    }
}

orc_sim *orc_create(const orc_cfg *cfg, const double *jc0_mult, const double *strain,
                    const double *c_wire) {
    return orc_create_ex(cfg, jc0_mult, strain, c_wire, 0);
}

orc_sim *orc_create_ex(const orc_cfg *cfg, const double *jc0_mult, const double *strain,
                       const double *c_wire, int field_only) {
    if (!cfg || !cfg_valid(cfg)) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->cfg = *cfg;
    const orc_cfg *c = &s->cfg;
    long N = 0, Nw = 0, nwe = 0;
    s->coil_off = (long *)calloc((size_t)c->n_coils + 1, sizeof(long));
    for (int ci = 0; ci < c->n_coils; ++ci) {
        s->coil_off[ci] = N;
        const long ne = c->ne[ci];
        N += (long)c->layers[ci] * c->turns[ci] * ne * ne;
        Nw += (long)c->layers[ci] * c->turns[ci];
        nwe += (long)c->layers[ci] * c->turns[ci] * ne * ne;
    }
    s->coil_off[c->n_coils] = N;
    s->N = N;
    s->Nw = Nw;
    s->r = dalloc(N); s->z = dalloc(N); s->d = dalloc(N); s->V = dalloc(N);
    s->coil = (int *)calloc((size_t)N, sizeof(int));
    s->wire = (int *)calloc((size_t)N, sizeof(int));
    s->wire_off = (long *)calloc((size_t)Nw + 1, sizeof(long));
    s->welem = (long *)calloc((size_t)nwe, sizeof(long));
    s->wn = (int *)calloc((size_t)Nw, sizeof(int));
    s->wcoil = (int *)calloc((size_t)Nw, sizeof(int));
    /* geometry (R1) */
    long w0 = 0, slot = 0;
    for (int ci = 0; ci < c->n_coils; ++ci) {
        const int ne = c->ne[ci], L = c->layers[ci], Tn = c->turns[ci];
        const long nz = (long)Tn * ne;
        const double ws = c->wire_side[ci], d = ws / ne;
        const double zbot = c->z_center[ci] - 0.5 * Tn * ws;
        for (int li = 0; li < L; ++li)
            for (int ti = 0; ti < Tn; ++ti) {
                const long w = w0 + (long)li * Tn + ti;
                s->wire_off[w] = slot;
                s->wn[w] = ne * ne;
                s->wcoil[w] = ci;
                for (int a = 0; a < ne; ++a)
                    for (int b = 0; b < ne; ++b) {
                        const long ir = (long)li * ne + a, iz = (long)ti * ne + b;
                        const long e = s->coil_off[ci] + ir * nz + iz;
                        s->welem[slot++] = e;
                        s->r[e] = c->r_inner[ci] + ((double)ir + 0.5) * d;
                        s->z[e] = zbot + ((double)iz + 0.5) * d;
                        s->d[e] = d;
                        s->V[e] = c->planar ? d * d : 2.0 * ORC_PI * s->r[e] * d * d;
                        s->coil[e] = ci;
                        s->wire[e] = (int)w;
                    }
            }
        w0 += (long)L * Tn;
    }
    s->wire_off[Nw] = slot;
    /* static part of Jc */
    s->jcs = dalloc(N);
    s->cw = dalloc(Nw);
    for (long e = 0; e < N; ++e) {
        const double mu = jc0_mult ? jc0_mult[e] : 1.0;
        const double ep = strain ? strain[e] : 0.0;
        s->jcs[e] = c->Jc0 * mu * (1.0 - c->eps_coef * pow(fabs(ep), c->eps_pow));
    }
    for (long w = 0; w < Nw; ++w) s->cw[w] = c_wire ? c_wire[w] : 1.0;
    /* per-wire inductance blocks (R2) */
    s->Mww = (double **)calloc((size_t)Nw, sizeof(double *));
    s->field_only = field_only;
    #pragma omp parallel for schedule(dynamic, 4)
    for (long w = 0; w < (field_only ? 0 : Nw); ++w) {
        const int n = s->wn[w];
        const long *el = s->welem + s->wire_off[w];
        double *M = dalloc((long)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const long ei = el[i], ej = el[j];
                M[i * n + j] = (i == j) ? orc_self_L(s->r[ei], s->d[ei])
                                        : orc_ring_M(s->r[ej], s->z[ej], s->r[ei], s->z[ei]);
            }
        s->Mww[w] = M;
    }
    /* coupling 1: each coil's full inductance matrix (public order inside the coil) */
    s->Mc = (double **)calloc((size_t)c->n_coils, sizeof(double *));
    for (int ci = 0; ci < c->n_coils && c->coupling == 1 && !field_only; ++ci) {
        const long o = s->coil_off[ci], n = s->coil_off[ci + 1] - o;
        double *M = dalloc(n * n);
        #pragma omp parallel for schedule(dynamic, 8)
        for (long i = 0; i < n; ++i)
            for (long j = 0; j < n; ++j)
                M[i * n + j] = (i == j) ? orc_self_L(s->r[o + i], s->d[o + i])
                                        : orc_ring_M(s->r[o + j], s->z[o + j], s->r[o + i], s->z[o + i]);
        s->Mc[ci] = M;
    }
    /* transport flux pattern (R3): flux through ring e per ampere of transport
       current carried uniformly by every other wire of the same coil */
    s->psi = dalloc(N);
    #pragma omp parallel for schedule(dynamic, 64)
    for (long e = 0; e < (field_only ? 0 : N); ++e) {
        const int ci = s->coil[e];
        nsum acc = {0.0, 0.0};
        for (long j = s->coil_off[ci]; j < s->coil_off[ci + 1]; ++j) {
            if (s->wire[j] == s->wire[e]) continue;
            ns_add(&acc, orc_ring_M(s->r[j], s->z[j], s->r[e], s->z[e]) / (double)s->wn[s->wire[j]]);
        }
        s->psi[e] = ns_val(&acc);
    }
    /* heat */
    s->nb = (long *)calloc((size_t)4 * N, sizeof(long));
    s->G = dalloc(4 * N);
    s->Gb = dalloc(N);
    build_heat(s);
    /* state */
    s->I = dalloc(N); s->u = dalloc(N); s->T = dalloc(N); s->Phi = dalloc(N);
    s->Br = dalloc(N); s->Bz = dalloc(N); s->E = dalloc(N); s->Ep = dalloc(N);
    s->Jc = dalloc(N); s->dI = dalloc(N); s->q = dalloc(N);
    s->Qw = dalloc(Nw); s->U = dalloc(Nw);
    s->onset = dalloc(Nw); s->quench = dalloc(Nw); s->Qon = dalloc(Nw);
    s->Qqu = dalloc(Nw); s->Tqu = dalloc(Nw); s->Pqu = dalloc(Nw);
    for (long w = 0; w < Nw; ++w) { s->onset[w] = -1.0; s->quench[w] = -1.0; }
    s->kmult = dalloc(N);
    for (long e = 0; e < N; ++e) s->kmult[e] = 1.0;
    s->IH = dalloc(N);
    s->emsub = dalloc(Nw);
    for (long e = 0; e < N; ++e) s->T[e] = c->T_bath;
    /* initial transport current I0 of each coil, spread evenly over the
       elements of each of its wires */
    for (long w = 0; w < Nw; ++w)
        for (int i = 0; i < s->wn[w]; ++i)
            s->I[s->welem[s->wire_off[w] + i]] = c->I0[s->wcoil[w]] / (double)s->wn[w];
    s->Tpeak = c->T_bath;
    s->Tpeak_e = -1;
    s->Tpeak_k = -1;
    return s;
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    if (s->Mww) for (long w = 0; w < s->Nw; ++w) free(s->Mww[w]);
    free(s->Mww);
    if (s->Mc) for (int ci = 0; ci < s->cfg.n_coils; ++ci) free(s->Mc[ci]);
    free(s->Mc);
    void *p[] = {s->r, s->z, s->d, s->V, s->coil, s->wire, s->coil_off, s->wire_off, s->welem,
                 s->wn, s->wcoil, s->jcs, s->cw, s->psi, s->nb, s->G, s->Gb, s->I, s->u, s->T,
                 s->Phi, s->Br, s->Bz, s->E, s->Ep, s->Jc, s->dI, s->q, s->Qw, s->U,
                 s->onset, s->quench, s->Qon, s->Qqu, s->Tqu, s->Pqu, s->kmult, s->IH, s->emsub};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(p[i]);
    free(s);
}

/* ------------------------------------------------------------------ */
/* field sum                                                           */
/* ------------------------------------------------------------------ */
static void field_at_element(const orc_sim *s, const double *I, long e, double *Br, double *Bz) {
    const int ci = s->coil[e];
    nsum ar = {0.0, 0.0}, az = {0.0, 0.0};
    for (long j = s->coil_off[ci]; j < s->coil_off[ci + 1]; ++j) {
        if (j == e || I[j] == 0.0) continue;
        double br, bz;
        orc_ring_B(s->r[j], s->z[j], s->r[e], s->z[e], I[j], &br, &bz);
        ns_add(&ar, br);
        ns_add(&az, bz);
    }
    *Br = ns_val(&ar);
    *Bz = ns_val(&az);
}

void orc_field_targets(const orc_sim *s, const double *I, long nt, const long *tgt,
                       double *Br, double *Bz) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < nt; ++i) field_at_element(s, I, tgt[i], &Br[i], &Bz[i]);
}

void orc_field_points(const orc_sim *s, const double *I, long np, const double *r,
                      const double *z, double *Br, double *Bz) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < np; ++i) {
        nsum ar = {0.0, 0.0}, az = {0.0, 0.0};
        for (long j = 0; j < s->N; ++j) {
            if (I[j] == 0.0) continue;
            double br, bz;
            orc_ring_B(s->r[j], s->z[j], r[i], z[i], I[j], &br, &bz);
            ns_add(&ar, br);
            ns_add(&az, bz);
        }
        Br[i] = ns_val(&ar);
        Bz[i] = ns_val(&az);
    }
}

int orc_wire_elems(const orc_sim *s, long w, long *dst) {
    if (w < 0 || w >= s->Nw) return 0;
    const int n = s->wn[w];
    for (int i = 0; i < n; ++i) dst[i] = s->welem[s->wire_off[w] + i];
    return n;
}

/* ------------------------------------------------------------------ */
/* dense Cholesky and triangular solves                                */
/* ------------------------------------------------------------------ */
static int cholesky(double *A, int n) { /* lower factor in place, row-major */
    for (int j = 0; j < n; ++j) {
        double dsum = A[j * n + j];
        for (int k = 0; k < j; ++k) dsum -= A[j * n + k] * A[j * n + k];
        if (!(dsum > 0.0)) return -1;
        const double ljj = sqrt(dsum);
        A[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / ljj;
        }
    }
    return 0;
}
static void chol_solve(const double *L, int n, double *x) { /* L L^T x = b in place */
    for (int i = 0; i < n; ++i) {
        double v = x[i];
        for (int k = 0; k < i; ++k) v -= L[i * n + k] * x[k];
        x[i] = v / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = x[i];
        for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
        x[i] = v / L[i * n + i];
    }
}

/* ------------------------------------------------------------------ */
/* coupled A-V solve (coupling = 1)                                    */
/* ------------------------------------------------------------------ */
/* Every ring e of a coil obeys 2 pi r_e E_e + U_w(e) = -dPhi_e/dt with the
   flux Phi_e = sum_j M_ej I_j + pi r_e^2 B_a of ALL element currents of the
   coil, and every wire carries the transport current.  Linearised backward
   Euler (E at I + dI is E + E' dI/d^2):
     A dI + dt P U = b,   P^T dI = dI_t 1,
     A = M + dt diag(2 pi r E'/d^2),  b = -pi r^2 dB_a - dt 2 pi r E,
   with P the element-to-wire incidence.  Solved per coil by a Cholesky
   factorisation of A: X = A^-1 b, Y = A^-1 P, then the loop voltages from
   (P^T Y) dt U = P^T X - dI_t 1 (the Schur complement, SPD), dI = X - Y dt U.
   The flux is updated as Phi += M dI + pi r^2 dB_a. */
static int coupled_solve(orc_sim *s, double dBa) {
    const orc_cfg *c = &s->cfg;
    const double dt = c->dt;
    int bad = 0;
    for (int ci = 0; ci < c->n_coils && !bad; ++ci) {
        const long o = s->coil_off[ci], n = s->coil_off[ci + 1] - o;
        const double dIt = c->ramp[ci] * dt;
        /* wires of the coil: the wire index of every element, local numbering */
        long w0 = -1, nw = 0;
        for (long w = 0; w < s->Nw; ++w)
            if (s->wcoil[w] == ci) { if (w0 < 0) w0 = w; ++nw; }
        double *A = dalloc(n * n), *X = dalloc(n), *Y = dalloc(n * nw), *S = dalloc(nw * nw);
        double *u = dalloc(nw), *MdI = dalloc(n);
        memcpy(A, s->Mc[ci], sizeof(double) * (size_t)(n * n));
        for (long i = 0; i < n; ++i) {
            const long e = o + i;
            const double d2 = s->d[e] * s->d[e];
            A[i * n + i] += dt * 2.0 * ORC_PI * s->r[e] * s->Ep[e] / d2;
            X[i] = -ORC_PI * s->r[e] * s->r[e] * dBa - dt * 2.0 * ORC_PI * s->r[e] * s->E[e];
        }
        if (cholesky(A, (int)n) != 0) { bad = 1; goto done; }
        chol_solve(A, (int)n, X);
        #pragma omp parallel for schedule(dynamic, 1)
        for (long v = 0; v < nw; ++v) {
            double *col = dalloc(n);
            for (long i = 0; i < n; ++i) col[i] = (s->wire[o + i] == w0 + v) ? 1.0 : 0.0;
            chol_solve(A, (int)n, col);
            for (long i = 0; i < n; ++i) Y[i * nw + v] = col[i];
            free(col);
        }
        for (long i = 0; i < n; ++i) {
            const long wi = s->wire[o + i] - w0;
            u[wi] += X[i];
            for (long v = 0; v < nw; ++v) S[wi * nw + v] += Y[i * nw + v];
        }
        for (long v = 0; v < nw; ++v) u[v] -= dIt;
        if (cholesky(S, (int)nw) != 0) { bad = 1; goto done; }
        chol_solve(S, (int)nw, u);  /* u = dt U */
        for (long v = 0; v < nw; ++v) s->U[w0 + v] = u[v] / dt;
        for (long i = 0; i < n; ++i) {
            double dI = X[i];
            for (long v = 0; v < nw; ++v) dI -= Y[i * nw + v] * u[v];
            s->dI[o + i] = dI;
        }
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            double v = 0.0;
            for (long j = 0; j < n; ++j) v += s->Mc[ci][i * n + j] * s->dI[o + j];
            MdI[i] = v;
        }
        for (long i = 0; i < n; ++i) {
            const long e = o + i;
            s->Phi[e] += MdI[i] + ORC_PI * s->r[e] * s->r[e] * dBa;
        }
    done:
        free(A); free(X); free(Y); free(S); free(u); free(MdI);
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* variable-step EM integration of a wire (em_tol > 0)                 */
/* ------------------------------------------------------------------ */
/* One linearised implicit Euler step of length h for wire w from the element
   currents of the step's state, with E and E' given per element (R5 with dt
   replaced by h): (M_ww + h diag(2 pi r E'/d^2)) dI + h U 1 = b, 1^T dI = ramp h,
   b = -ramp h Psi_u - pi r^2 dBa/dt h - h 2 pi r E.  Returns nonzero if the
   factorisation fails. */
static int be_step(const orc_sim *s, long w, double h, const double *E, const double *Ep, double *dI,
                   double *U) {
    const orc_cfg *c = &s->cfg;
    const int n = s->wn[w];
    const double dIt = c->ramp[s->wcoil[w]] * h, dBa = c->dBa_dt * h;
    const long *el = s->welem + s->wire_off[w];
    double *A = dalloc((long)n * n), *y = dalloc(n);
    memcpy(A, s->Mww[w], sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) {
        const long e = el[i];
        const double d2 = s->d[e] * s->d[e];
        A[i * n + i] += h * 2.0 * ORC_PI * s->r[e] * Ep[i] / d2;
        dI[i] = -dIt * s->psi[e] - ORC_PI * s->r[e] * s->r[e] * dBa - h * 2.0 * ORC_PI * s->r[e] * E[i];
        y[i] = 1.0;
    }
    int bad = cholesky(A, n);
    if (!bad) {
        chol_solve(A, n, dI);
        chol_solve(A, n, y);
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < n; ++i) { sx += dI[i]; sy += y[i]; }
        *U = (sx - dIt) / (h * sy);
        for (int i = 0; i < n; ++i) dI[i] -= h * (*U) * y[i];
    }
    free(A); free(y);
    return bad;
}

/* The wire's currents over [t_k, t_k + dt] with B^k and T^k (so Jc) held, as
   the paper integrates the electromagnetic equations with a variable time
   step to follow the stiff power law (Methods, Numerical Algorithm, last
   sentence).  Substeps h = dt / 2^m.  An attempt takes one step of h and two
   of h/2 from the same currents I (E, E' re-evaluated at the midpoint
   currents); with I1 and I2 the two results,
     err = max_e |I2_e - I1_e| / (em_tol max(|I2_e|, Jc_e d^2)),
   err <= 1 keeps the extrapolated 2 I2 - I1 (second order; the extrapolated
   linearly implicit Euler step is L-stable) and advances by h, otherwise m
   grows by one and the attempt is repeated (at the finest level the attempt
   is kept whatever err).  After a kept substep with err <= 1/4, at a position
   that is a multiple of 2h, m falls by one.  Every step starts at m = 0.  Per
   kept substep the Joule source R8 of each half step, E_lin J^{new}, is
   accumulated times its length, and the loop voltage as 2 U2 - U1 (U2 the
   mean of the half steps'); q and U_w are their averages over dt.  dI is the
   step's total change; the flux update is that of R4 with it. */
static int em_wire(orc_sim *s, long w) {
    const orc_cfg *c = &s->cfg;
    const int n = s->wn[w];
    const long *el = s->welem + s->wire_off[w];
    const int L = c->em_max_level > 0 ? c->em_max_level : 10;
    const long full = 1L << L;
    double *Iv = dalloc(n), *Im = dalloc(n), *E1 = dalloc(n), *P1 = dalloc(n), *Em = dalloc(n), *Pm = dalloc(n);
    double *d1 = dalloc(n), *da = dalloc(n), *db = dalloc(n), *qa = dalloc(n);
    double Uacc = 0.0, x;
    long pos = 0;
    int m = 0, nsub = 0, bad = 0;
    for (int i = 0; i < n; ++i) Iv[i] = s->I[el[i]];
    while (pos < full && !bad) {
        const double h = ldexp(c->dt, -m);
        double U1, Ua, Ub;
        for (int i = 0; i < n; ++i) {
            const long e = el[i];
            bad |= local_EJ(c, Iv[i] / (s->d[e] * s->d[e]), s->Jc[e], &E1[i], &P1[i], &x);
        }
        if (bad) break;
        bad |= be_step(s, w, h, E1, P1, d1, &U1);
        bad |= be_step(s, w, 0.5 * h, E1, P1, da, &Ua);
        for (int i = 0; i < n; ++i) {
            const long e = el[i];
            Im[i] = Iv[i] + da[i];
            bad |= local_EJ(c, Im[i] / (s->d[e] * s->d[e]), s->Jc[e], &Em[i], &Pm[i], &x);
        }
        if (bad) break;
        bad |= be_step(s, w, 0.5 * h, Em, Pm, db, &Ub);
        if (bad) break;
        double err = 0.0;
        for (int i = 0; i < n; ++i) {
            const long e = el[i];
            const double d2 = s->d[e] * s->d[e];
            const double I2 = Im[i] + db[i], I1 = Iv[i] + d1[i];
            const double sc = c->em_tol * fmax(fabs(I2), s->Jc[e] > 0.0 ? s->Jc[e] * d2 : 0.0);
            const double dif = fabs(I2 - I1);
            const double ei = (sc > 0.0) ? dif / sc : (dif == 0.0 ? 0.0 : INFINITY);
            if (ei > err) err = ei;
        }
        if (err > 1.0 && m < L) {
            ++m;
            continue;
        }
        for (int i = 0; i < n; ++i) {
            const long e = el[i];
            const double d2 = s->d[e] * s->d[e];
            const double I2 = Im[i] + db[i];
            const double Ea = E1[i] + P1[i] * da[i] / d2, Eb = Em[i] + Pm[i] * db[i] / d2;
            qa[i] += 0.5 * h * (Ea * (Im[i] / d2) + Eb * (I2 / d2));
            Iv[i] = 2.0 * I2 - (Iv[i] + d1[i]);
        }
        Uacc += h * (Ua + Ub - U1);
        pos += 1L << (L - m);
        ++nsub;
        if (err <= 0.25 && m > 0 && pos % (1L << (L - m + 1)) == 0) --m;
    }
    if (!bad) {
        const double dt = c->dt;
        for (int i = 0; i < n; ++i) {
            const long e = el[i];
            s->dI[e] = Iv[i] - s->I[e];
            s->q[e] = qa[i] / dt;
        }
        s->U[w] = Uacc / dt;
        s->emsub[w] = (double)nsub;
    }
    free(Iv); free(Im); free(E1); free(P1); free(Em); free(Pm); free(d1); free(da); free(db); free(qa);
    return bad;
}

/* ------------------------------------------------------------------ */
/* subelement model (subelements >= 1)                                 */
/* ------------------------------------------------------------------ */
/* Per wire, with A = M_ww + dt diag(2 pi r E'/d^2) and rho_e = E_e / J_e
   (E'_e where J_e = 0):
     A dI_H = b_H - dt P_s U_s,  P_s^T dI_H = 0   (one loop voltage per subelement)
     A dI_I = b_I - dt 1 U_w,    1^T dI_I = dI_t  (one loop voltage per wire)
     b_H = -dI_t Psi_u - pi r^2 dB_a - dt 2 pi r rho J_H,  b_I = -dt 2 pi r rho J_I,
   P_s the element-to-subelement incidence.  b_H + b_I is the drive of the
   one-subelement model, so with s = 1 the sum dI_H + dI_I is its solution.
   dI = dI_H + dI_I; I_H += dI_H; the flux and Joule source as for the
   wire model.  An element of subelement s sees the loop voltage U_w + U_s;
   the wire's voltage is their average over its (equal) elements,
   U_w + mean_s U_s, which is the wire model's U when s = 1. */
static int subelement_solve(orc_sim *s, double dBa) {
    const orc_cfg *c = &s->cfg;
    const double dt = c->dt;
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 4)
    for (long w = 0; w < s->Nw; ++w) {
        const int n = s->wn[w];
        const int ci = s->wcoil[w];
        const int ne = c->ne[ci], sb = ne / c->subelements, ns = c->subelements * c->subelements;
        const double dIt = c->ramp[ci] * dt;
        const long *el = s->welem + s->wire_off[w];
        double *A = dalloc((long)n * n), *xh = dalloc(n), *xi = dalloc(n), *y = dalloc(n);
        double *Y = dalloc((long)n * ns), *S = dalloc((long)ns * ns), *u = dalloc(ns), *col = dalloc(n);
        int *sub = (int *)calloc((size_t)n, sizeof(int));
        memcpy(A, s->Mww[w], sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; ++i) {
            const long e = el[i];
            const double d2 = s->d[e] * s->d[e];
            const double J = s->I[e] / d2, JH = s->IH[e] / d2;
            const double rho = (J != 0.0) ? s->E[e] / J : s->Ep[e];
            A[i * n + i] += dt * 2.0 * ORC_PI * s->r[e] * s->Ep[e] / d2;
            xh[i] = -dIt * s->psi[e] - ORC_PI * s->r[e] * s->r[e] * dBa - dt * 2.0 * ORC_PI * s->r[e] * rho * JH;
            xi[i] = -dt * 2.0 * ORC_PI * s->r[e] * rho * (J - JH);
            y[i] = 1.0;
            /* local element order a*ne + b inside the wire: subelement of (a, b) */
            sub[i] = ((i / ne) / sb) * c->subelements + (i % ne) / sb;
        }
        if (cholesky(A, n) != 0) {
            #pragma omp atomic write
            bad = 1;
        } else {
            chol_solve(A, n, xh);
            chol_solve(A, n, xi);
            chol_solve(A, n, y);
            for (int v = 0; v < ns; ++v) {
                for (int i = 0; i < n; ++i) col[i] = (sub[i] == v) ? 1.0 : 0.0;
                chol_solve(A, n, col);
                for (int i = 0; i < n; ++i) Y[(long)i * ns + v] = col[i];
            }
            for (int i = 0; i < n; ++i) {
                u[sub[i]] += xh[i];
                for (int v = 0; v < ns; ++v) S[sub[i] * ns + v] += Y[(long)i * ns + v];
            }
            if (cholesky(S, ns) != 0) {
                #pragma omp atomic write
                bad = 1;
            } else {
                chol_solve(S, ns, u);  /* dt U_s */
                double sx = 0.0, sy = 0.0;
                for (int i = 0; i < n; ++i) { sx += xi[i]; sy += y[i]; }
                const double U = (sx - dIt) / (dt * sy);
                double uh = 0.0;
                for (int v = 0; v < ns; ++v) uh += u[v];
                /* wire voltage: the element-averaged loop voltage U_I + mean_s U_s */
                s->U[w] = U + uh / ((double)ns * dt);
                for (int i = 0; i < n; ++i) {
                    double dIH = xh[i];
                    for (int v = 0; v < ns; ++v) dIH -= Y[(long)i * ns + v] * u[v];
                    s->dI[el[i]] = dIH + (xi[i] - dt * U * y[i]);
                    s->IH[el[i]] += dIH;
                }
                for (int i = 0; i < n; ++i) {
                    double v = 0.0;
                    for (int j = 0; j < n; ++j) v += s->Mww[w][i * n + j] * s->dI[el[j]];
                    col[i] = v;
                }
                for (int i = 0; i < n; ++i) {
                    const long e = el[i];
                    s->Phi[e] += col[i] + dIt * s->psi[e] + ORC_PI * s->r[e] * s->r[e] * dBa;
                }
            }
        }
        free(A); free(xh); free(xi); free(y); free(Y); free(S); free(u); free(col); free(sub);
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* ADI heat step (heat_solver = 1)                                     */
/* ------------------------------------------------------------------ */
/* Peaceman-Rachford alternating-direction implicit step on the finite
   volumes (paper, Methods, heat paragraph: ADI on the composite coil, with
   c, kappa and h proportional to T^3).  Coefficients frozen at T^n:
   C = dU/dT, k_e = k0 (T_e/T_ref)^k_exp kmult_e, h_e = h0 (T_e/T_ref)^h_exp;
   face conductance G_ef = A / (d/(2 k_e) + d/(2 k_f) + R_ef), R_ef the
   insulation resistance ins_R0 (T_ref / T_face)^k_exp, T_face = (T_e + T_f)/2,
   on faces between different wires; border G^b = A / (1/h_e + d/(2 k_e)).
   With L_r, L_z the radial and axial parts of the net inflow (borders
   included) and q held fixed:
     V C (T* - T^n) / (dt/2)  = L_r(T*)  + L_z(T^n) + V q   (tridiagonal in r)
     V C (T** - T*) / (dt/2)  = L_r(T*)  + L_z(T**) + V q   (tridiagonal in z)
   and the enthalpy takes the inflow of those two half steps,
     u^{n+1} = u^n + (dt/V) [L_r(T*) + (L_z(T^n) + L_z(T**))/2] + dt q,
   T^{n+1} = T(u^{n+1}), so that interior fluxes cancel and the energy balance
   is exact.  Tridiagonal systems by the Thomas algorithm. */
static double k_at(const orc_sim *s, long e, double T) {
    const orc_cfg *c = &s->cfg;
    return c->k0 * pow(T / c->T_ref, c->k_exp) * s->kmult[e];
}

static double face_G(const orc_sim *s, long e, long f, double area, const double *T) {
    const orc_cfg *c = &s->cfg;
    const double d = s->d[e];
    double R = d / (2.0 * k_at(s, e, T[e])) + d / (2.0 * k_at(s, f, T[f]));
    if (c->ins_R0 > 0.0 && s->wire[e] != s->wire[f])
        R += c->ins_R0 * pow(c->T_ref / (0.5 * (T[e] + T[f])), c->k_exp);
    return area / R;
}

static double border_G(const orc_sim *s, long e, double area, const double *T) {
    const orc_cfg *c = &s->cfg;
    if (!(c->h0 > 0.0)) return 0.0;
    const double h = c->h0 * pow(T[e] / c->T_ref, c->h_exp);
    return area / (1.0 / h + s->d[e] / (2.0 * k_at(s, e, T[e])));
}

static void thomas(long n, const double *a, const double *b, const double *cc, const double *r, double *x,
                   double *cp, double *dp) {
    /* a_i x_{i-1} + b_i x_i + c_i x_{i+1} = r_i */
    cp[0] = cc[0] / b[0];
    dp[0] = r[0] / b[0];
    for (long i = 1; i < n; ++i) {
        const double m = b[i] - a[i] * cp[i - 1];
        cp[i] = cc[i] / m;
        dp[i] = (r[i] - a[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (long i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

static void heat_adi(orc_sim *s) {
    const orc_cfg *c = &s->cfg;
    const long N = s->N;
    const double dt = c->dt;
    double *Tn = dalloc(N), *Ts = dalloc(N), *Tss = dalloc(N), *Cv = dalloc(N);
    double *Gf = dalloc(4 * N), *Gbr = dalloc(N), *Gbz = dalloc(N), *Lz0 = dalloc(N), *Lr1 = dalloc(N);
    memcpy(Tn, s->T, sizeof(double) * (size_t)N);
    /* coefficients at T^n; faces 0 inner, 1 outer (radial), 2 lower, 3 upper (axial) */
    for (long e = 0; e < N; ++e) {
        const int ci = s->coil[e];
        const double d = s->d[e];
        const long ir = (long)((s->r[e] - c->r_inner[ci]) / d);
        const double rin = c->r_inner[ci];
        double area[4];
        if (c->planar) {
            area[0] = area[1] = area[2] = area[3] = d;
        } else {
            area[0] = 2.0 * ORC_PI * (rin + (double)ir * d) * d;
            area[1] = 2.0 * ORC_PI * (rin + (double)(ir + 1) * d) * d;
            area[2] = area[3] = 2.0 * ORC_PI * s->r[e] * d;
        }
        Cv[e] = s->V[e] * c->C0 * pow(Tn[e] / c->T_ref, c->cp_exp);
        Gbr[e] = Gbz[e] = 0.0;
        for (int f = 0; f < 4; ++f) {
            const long nbr = s->nb[4 * e + f];
            if (nbr >= 0) {
                Gf[4 * e + f] = face_G(s, e, nbr, area[f], Tn);
            } else {
                Gf[4 * e + f] = 0.0;
                if (f < 2) Gbr[e] += border_G(s, e, area[f], Tn);
                else       Gbz[e] += border_G(s, e, area[f], Tn);
            }
        }
        double lz = Gbz[e] * (c->T_bath - Tn[e]);
        for (int f = 2; f < 4; ++f) {
            const long nbr = s->nb[4 * e + f];
            if (nbr >= 0) lz += Gf[4 * e + f] * (Tn[nbr] - Tn[e]);
        }
        Lz0[e] = lz;
    }
    /* half step 1: implicit in r, one system per coil column */
    for (int ci = 0; ci < c->n_coils; ++ci) {
        const long o = s->coil_off[ci];
        const long nr = (long)c->layers[ci] * c->ne[ci], nz = (long)c->turns[ci] * c->ne[ci];
        double *a = dalloc(nr), *b = dalloc(nr), *cc = dalloc(nr), *rr = dalloc(nr), *x = dalloc(nr);
        double *cp = dalloc(nr), *dp = dalloc(nr);
        for (long iz = 0; iz < nz; ++iz) {
            for (long ir = 0; ir < nr; ++ir) {
                const long e = o + ir * nz + iz;
                const double m = 2.0 * Cv[e] / dt;
                a[ir] = -Gf[4 * e + 0];
                cc[ir] = -Gf[4 * e + 1];
                b[ir] = m + Gf[4 * e + 0] + Gf[4 * e + 1] + Gbr[e];
                rr[ir] = m * Tn[e] + Lz0[e] + s->V[e] * s->q[e] + Gbr[e] * c->T_bath;
            }
            thomas(nr, a, b, cc, rr, x, cp, dp);
            for (long ir = 0; ir < nr; ++ir) Ts[o + ir * nz + iz] = x[ir];
        }
        free(a); free(b); free(cc); free(rr); free(x); free(cp); free(dp);
    }
    for (long e = 0; e < N; ++e) {
        double lr = Gbr[e] * (c->T_bath - Ts[e]);
        for (int f = 0; f < 2; ++f) {
            const long nbr = s->nb[4 * e + f];
            if (nbr >= 0) lr += Gf[4 * e + f] * (Ts[nbr] - Ts[e]);
        }
        Lr1[e] = lr;
    }
    /* half step 2: implicit in z, one system per coil row */
    for (int ci = 0; ci < c->n_coils; ++ci) {
        const long o = s->coil_off[ci];
        const long nr = (long)c->layers[ci] * c->ne[ci], nz = (long)c->turns[ci] * c->ne[ci];
        double *a = dalloc(nz), *b = dalloc(nz), *cc = dalloc(nz), *rr = dalloc(nz), *x = dalloc(nz);
        double *cp = dalloc(nz), *dp = dalloc(nz);
        for (long ir = 0; ir < nr; ++ir) {
            for (long iz = 0; iz < nz; ++iz) {
                const long e = o + ir * nz + iz;
                const double m = 2.0 * Cv[e] / dt;
                a[iz] = -Gf[4 * e + 2];
                cc[iz] = -Gf[4 * e + 3];
                b[iz] = m + Gf[4 * e + 2] + Gf[4 * e + 3] + Gbz[e];
                rr[iz] = m * Ts[e] + Lr1[e] + s->V[e] * s->q[e] + Gbz[e] * c->T_bath;
            }
            thomas(nz, a, b, cc, rr, x, cp, dp);
            for (long iz = 0; iz < nz; ++iz) Tss[o + ir * nz + iz] = x[iz];
        }
        free(a); free(b); free(cc); free(rr); free(x); free(cp); free(dp);
    }
    /* enthalpy from the half steps' inflow, border outflow */
    nsum out = {0.0, 0.0};
    for (long e = 0; e < N; ++e) {
        double lz = Gbz[e] * (c->T_bath - Tss[e]);
        for (int f = 2; f < 4; ++f) {
            const long nbr = s->nb[4 * e + f];
            if (nbr >= 0) lz += Gf[4 * e + f] * (Tss[nbr] - Tss[e]);
        }
        s->u[e] += dt / s->V[e] * (Lr1[e] + 0.5 * (Lz0[e] + lz)) + dt * s->q[e];
        s->T[e] = T_of_u(c, s->u[e]);
        ns_add(&out, dt * (Gbr[e] * (Ts[e] - c->T_bath) + 0.5 * Gbz[e] * ((Tn[e] - c->T_bath) + (Tss[e] - c->T_bath))));
    }
    s->Qout += ns_val(&out);
    free(Tn); free(Ts); free(Tss); free(Cv); free(Gf); free(Gbr); free(Gbz); free(Lz0); free(Lr1);
}

/* ------------------------------------------------------------------ */
/* one time step                                                       */
/* ------------------------------------------------------------------ */
int orc_step(orc_sim *s) {
    if (s->field_only) return -1;
    const orc_cfg *c = &s->cfg;
    const long N = s->N, Nw = s->Nw;
    const double dt = c->dt;
    const double tk = (double)s->step * dt;
    const double Ba = c->dBa_dt * tk;
    const double dBa = c->dBa_dt * dt;
    int bad = 0;

    /* 1. field from the element currents at step k */
    #pragma omp parallel for schedule(dynamic, 16)
    for (long e = 0; e < N; ++e) {
        double br, bz;
        field_at_element(s, s->I, e, &br, &bz);
        s->Br[e] = br;
        s->Bz[e] = bz + Ba;
    }

    /* 2. local law at step k */
    double maxx = 0.0;
    for (long e = 0; e < N; ++e) {
        const double d2 = s->d[e] * s->d[e];
        const double J = s->I[e] / d2;
        const double Bm = sqrt(s->Br[e] * s->Br[e] + s->Bz[e] * s->Bz[e]);
        const double fT = fmax(0.0, 1.0 - s->T[e] / c->Tc);
        const double Jc = s->cw[s->wire[e]] * s->jcs[e] * fT * c->B0 / (c->B0 + Bm);
        s->Jc[e] = Jc;
        double x;
        if (local_EJ(c, J, Jc, &s->E[e], &s->Ep[e], &x)) bad = 1;
        if (x > maxx) maxx = x;
    }

    /* flux-jump onset (|J/Jc| > 1) and quench (rho > 0.95 rho_n) of each wire,
       from the local law of this step (paper, Results: flux jumps and quenches
       propagation in a coil) */
    for (long w = 0; w < Nw; ++w) {
        const long *el = s->welem + s->wire_off[w];
        double xw = 0.0, sEJ = 0.0, sJJ = 0.0, sV = 0.0, Tw = -INFINITY;
        for (int i = 0; i < s->wn[w]; ++i) {
            const long e = el[i];
            const double d2 = s->d[e] * s->d[e];
            const double J = s->I[e] / d2;
            const double x = (J == 0.0) ? 0.0 : (s->Jc[e] > 0.0 ? fabs(J) / s->Jc[e] : INFINITY);
            if (x > xw) xw = x;
            sEJ += s->V[e] * s->E[e] * J;
            sJJ += s->V[e] * J * J;
            sV += s->V[e];
            if (s->T[e] > Tw) Tw = s->T[e];
        }
        if (s->onset[w] < 0.0 && xw > 1.0) {
            s->onset[w] = (double)s->step;
            s->Qon[w] = s->Qw[w];
        }
        if (c->rho_n > 0.0 && s->quench[w] < 0.0 && sJJ > 0.0 && sEJ / sJJ > 0.95 * c->rho_n) {
            s->quench[w] = (double)s->step;
            s->Qqu[w] = s->Qw[w];
            s->Tqu[w] = Tw;
            s->Pqu[w] = sEJ / sV;
        }
    }

    /* 3. A-V solve, linearised backward Euler */
    if (c->coupling == 1 && coupled_solve(s, dBa)) return -4;
    if (c->subelements >= 1 && subelement_solve(s, dBa)) return -4;
    #pragma omp parallel for schedule(dynamic, 4)
    for (long w = 0; w < ((c->coupling == 1 || c->subelements >= 1) ? 0 : Nw); ++w) {
        const int n = s->wn[w];
        const int ci = s->wcoil[w];
        const double dIt = c->ramp[ci] * dt;
        const long *el = s->welem + s->wire_off[w];
        double *A = dalloc((long)n * n), *x = dalloc(n), *y = dalloc(n), *MdI = dalloc(n);
        s->emsub[w] = 1.0;
        if (c->em_tol > 0.0) {
            /* variable-step integration: dI, q and U_w from the substeps */
            if (em_wire(s, w)) {
                #pragma omp atomic write
                bad = 1;
            } else {
                for (int i = 0; i < n; ++i) {
                    double v = 0.0;
                    for (int j = 0; j < n; ++j) v += s->Mww[w][i * n + j] * s->dI[el[j]];
                    MdI[i] = v;
                }
                for (int i = 0; i < n; ++i) {
                    const long e = el[i];
                    s->Phi[e] += MdI[i] + dIt * s->psi[e] + ORC_PI * s->r[e] * s->r[e] * dBa;
                }
            }
            free(A); free(x); free(y); free(MdI);
            continue;
        }
        memcpy(A, s->Mww[w], sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; ++i) {
            const long e = el[i];
            const double d2 = s->d[e] * s->d[e];
            A[i * n + i] += dt * 2.0 * ORC_PI * s->r[e] * s->Ep[e] / d2;
            x[i] = -dIt * s->psi[e] - ORC_PI * s->r[e] * s->r[e] * dBa
                   - dt * 2.0 * ORC_PI * s->r[e] * s->E[e];
            y[i] = 1.0;
        }
        if (cholesky(A, n) != 0) {
            #pragma omp atomic write
            bad = 1;
        } else {
            chol_solve(A, n, x);
            chol_solve(A, n, y);
            double sx = 0.0, sy = 0.0;
            for (int i = 0; i < n; ++i) { sx += x[i]; sy += y[i]; }
            const double U = (sx - dIt) / (dt * sy);
            s->U[w] = U;
            for (int i = 0; i < n; ++i) s->dI[el[i]] = x[i] - dt * U * y[i];
            /* flux update Phi += M_ww dI + dI_t Psi_u + pi r^2 dB_a */
            for (int i = 0; i < n; ++i) {
                double v = 0.0;
                for (int j = 0; j < n; ++j) v += s->Mww[w][i * n + j] * s->dI[el[j]];
                MdI[i] = v;
            }
            for (int i = 0; i < n; ++i) {
                const long e = el[i];
                s->Phi[e] += MdI[i] + dIt * s->psi[e] + ORC_PI * s->r[e] * s->r[e] * dBa;
            }
        }
        free(A); free(x); free(y); free(MdI);
    }
    if (bad) return -4;

    /* currents, Joule source q = E_lin J^{k+1} (R8), Q accumulation */
    nsum qsum = {0.0, 0.0};
    for (long w = 0; w < Nw; ++w) {
        const long *el = s->welem + s->wire_off[w];
        nsum qw = {0.0, 0.0};
        for (int i = 0; i < s->wn[w]; ++i) {
            const long e = el[i];
            const double d2 = s->d[e] * s->d[e];
            s->I[e] += s->dI[e];
            if (c->em_tol <= 0.0) {  /* else q is the substeps' average */
                const double Elin = s->E[e] + s->Ep[e] * s->dI[e] / d2;
                s->q[e] = Elin * (s->I[e] / d2);
            }
            ns_add(&qw, dt * s->V[e] * s->q[e]);
        }
        s->Qw[w] += ns_val(&qw);
        ns_add(&qsum, ns_val(&qw));
    }
    s->Q += ns_val(&qsum);
    {
        nsum us = {0.0, 0.0};
        for (long w = 0; w < Nw; ++w) ns_add(&us, s->U[w]);
        s->sumU = ns_val(&us);
    }
    s->maxx = maxx;

    /* 4. heat: ADI, or explicit with n_sub substeps, q held fixed */
    if (c->heat_solver == 1) heat_adi(s);
    const double hs = dt / (double)s->n_sub;
    double *un = dalloc(N);
    for (int sub = 0; sub < (c->heat_solver == 1 ? 0 : s->n_sub); ++sub) {
        nsum out = {0.0, 0.0};
        for (long e = 0; e < N; ++e) {
            double flux = s->Gb[e] * (c->T_bath - s->T[e]);
            for (int f = 0; f < 4; ++f) {
                const long nbr = s->nb[4 * e + f];
                if (nbr >= 0) flux += s->G[4 * e + f] * (s->T[nbr] - s->T[e]);
            }
            un[e] = s->u[e] + hs / s->V[e] * flux + hs * s->q[e];
            ns_add(&out, hs * s->Gb[e] * (s->T[e] - c->T_bath));
        }
        s->Qout += ns_val(&out);
        for (long e = 0; e < N; ++e) {
            s->u[e] = un[e];
            s->T[e] = T_of_u(c, un[e]);
        }
    }
    free(un);

    /* 5. peak temperature, lowest (step, element) on ties */
    for (long e = 0; e < N; ++e) {
        if (!isfinite(s->T[e]) || !isfinite(s->I[e])) bad = 1;
        if (s->T[e] > s->Tpeak) {
            s->Tpeak = s->T[e];
            s->Tpeak_e = e;
            s->Tpeak_k = s->step + 1;
        }
    }
    s->step += 1;
    return bad ? -4 : 0;
}

int orc_run(orc_sim *s, long nsteps) {
    for (long k = 0; k < nsteps; ++k) {
        const int rc = orc_step(s);
        if (rc) return rc;
    }
    return 0;
}

int orc_get(const orc_sim *s, int field, double *dst, long count) {
    const long N = s->N, Nw = s->Nw;
    const double *src = NULL;
    long n = N;
    switch (field) {
        case ORC_I: src = s->I; break;
        case ORC_BR: src = s->Br; break;
        case ORC_BZ: src = s->Bz; break;
        case ORC_T: src = s->T; break;
        case ORC_PHI: src = s->Phi; break;
        case ORC_QW: src = s->Qw; n = Nw; break;
        case ORC_UW: src = s->U; n = Nw; break;
        case ORC_E: src = s->E; break;
        case ORC_EP: src = s->Ep; break;
        case ORC_U: src = s->u; break;
        case ORC_Q: src = s->q; break;
        case ORC_PSI: src = s->psi; break;
        case ORC_R: src = s->r; break;
        case ORC_Z: src = s->z; break;
        case ORC_V: src = s->V; break;
        case ORC_JC: src = s->Jc; break;
        case ORC_DI: src = s->dI; break;
        case ORC_ONSET: src = s->onset; n = Nw; break;
        case ORC_QUENCH: src = s->quench; n = Nw; break;
        case ORC_Q_ONSET: src = s->Qon; n = Nw; break;
        case ORC_Q_QUENCH: src = s->Qqu; n = Nw; break;
        case ORC_T_QUENCH: src = s->Tqu; n = Nw; break;
        case ORC_P_QUENCH: src = s->Pqu; n = Nw; break;
        case ORC_KMULT: src = s->kmult; break;
        case ORC_IH: src = s->IH; break;
        case ORC_EMSUB: src = s->emsub; n = Nw; break;
        case ORC_J:
            if (count < N) return -1;
            for (long e = 0; e < N; ++e) dst[e] = s->I[e] / (s->d[e] * s->d[e]);
            return 0;
        default: return -1;
    }
    if (count < n) return -1;
    memcpy(dst, src, sizeof(double) * (size_t)n);
    return 0;
}

int orc_set(orc_sim *s, int field, const double *src, long count) {
    const long N = s->N;
    if (count < N) return -1;
    switch (field) {
        case ORC_I: memcpy(s->I, src, sizeof(double) * (size_t)N); return 0;
        case ORC_T:
            for (long e = 0; e < N; ++e) { s->T[e] = src[e]; s->u[e] = u_of_T(&s->cfg, src[e]); }
            return 0;
        case ORC_KMULT:
            for (long e = 0; e < N; ++e) if (!(src[e] > 0.0) || !isfinite(src[e])) return -1;
            memcpy(s->kmult, src, sizeof(double) * (size_t)N);
            return 0;
        default: return -1;
    }
}

int orc_scalars(const orc_sim *s, double *dst, int n) {
    double v[12];
    v[0] = (double)s->step * s->cfg.dt;
    v[1] = (double)s->step;
    v[2] = s->Q;
    v[3] = s->Tpeak;
    v[4] = s->sumU;
    v[5] = s->maxx;
    v[6] = s->Qout;
    {
        nsum st = {0.0, 0.0};
        for (long e = 0; e < s->N; ++e) ns_add(&st, s->V[e] * s->u[e]);
        v[7] = ns_val(&st);
    }
    v[8] = s->cfg.I0[0] + s->cfg.ramp[0] * v[0];
    v[9] = (double)s->Tpeak_e;
    v[10] = (double)s->Tpeak_k;
    v[11] = (double)s->n_sub;
    for (int i = 0; i < n && i < 12; ++i) dst[i] = v[i];
    return 0;
}

/* ------------------------------------------------------------------ */
/* tangent-linear model (forward-mode derivative of the step)          */
/* ------------------------------------------------------------------ */
/* Differentiates the same discrete step along a direction in the per-wire Jc
   multipliers c_w and the per-coil ramp rates.  The primal step is
   orc_step(); the tangent lines below use its intermediate values (B^k, Jc,
   E, E', dI at step k) and re-derive the heat substep temperatures.
   Non-smooth points take the zero branch: |B| = 0, T >= Tc, J = 0.  The peak
   temperature's derivative is that of the element and step where the peak was
   last raised. */
int orc_tangent(const orc_cfg *cfg, const double *jc0_mult, const double *strain,
                const double *c_wire, const double *dc_wire, const double *dramp,
                long nsteps, double *obj, double *dobj) {
    if (cfg->coupling != 0 || cfg->heat_solver != 0 || cfg->subelements >= 1 || cfg->em_tol > 0.0) return -1;
    orc_sim *s = orc_create(cfg, jc0_mult, strain, c_wire);
    if (!s) return -1;
    const orc_cfg *c = &s->cfg;
    const long N = s->N, Nw = s->Nw;
    const double dt = c->dt;
    const double hs = dt / (double)s->n_sub;
    double *dI = dalloc(N), *du = dalloc(N), *Ik = dalloc(N), *Tk = dalloc(N), *uk = dalloc(N);
    double *dBr = dalloc(N), *dBz = dalloc(N), *dE = dalloc(N), *dEp = dalloc(N), *ddI = dalloc(N);
    double *dq = dalloc(N), *Tsub = dalloc(N), *usub = dalloc(N), *dTsub = dalloc(N);
    double *unew = dalloc(N), *dunew = dalloc(N);
    double dQ = 0.0, dTpeak = 0.0;
    int rc = 0;
    for (long k = 0; k < nsteps && rc == 0; ++k) {
        memcpy(Ik, s->I, sizeof(double) * (size_t)N);
        memcpy(Tk, s->T, sizeof(double) * (size_t)N);
        memcpy(uk, s->u, sizeof(double) * (size_t)N);
        rc = orc_step(s);
        if (rc) break;
        /* 1. field tangent */
        #pragma omp parallel for schedule(dynamic, 16)
        for (long e = 0; e < N; ++e) field_at_element(s, dI, e, &dBr[e], &dBz[e]);
        /* 2. local law tangent at step k */
        for (long e = 0; e < N; ++e) {
            const double d2 = s->d[e] * s->d[e];
            const double J = Ik[e] / d2;
            dE[e] = 0.0;
            dEp[e] = 0.0;
            if (J == 0.0 && !(c->rho_n > 0.0)) continue;
            const double Br = s->Br[e], Bz = s->Bz[e];
            const double Bm = sqrt(Br * Br + Bz * Bz);
            const double dBm = Bm > 0.0 ? (Br * dBr[e] + Bz * dBz[e]) / Bm : 0.0;
            const double Ck = c->C0 * pow(Tk[e] / c->T_ref, c->cp_exp);
            const double dT = du[e] / Ck;
            const double fT = fmax(0.0, 1.0 - Tk[e] / c->Tc);
            const double dfT = (Tk[e] < c->Tc) ? -dT / c->Tc : 0.0;
            const double fB = c->B0 / (c->B0 + Bm);
            const double dfB = -c->B0 / ((c->B0 + Bm) * (c->B0 + Bm)) * dBm;
            const int w = s->wire[e];
            const double Jc = s->Jc[e];
            const double dJc = (dc_wire ? dc_wire[w] : 0.0) * s->jcs[e] * fT * fB
                             + s->cw[w] * s->jcs[e] * (dfT * fB + fT * dfB);
            local_EJ_tangent(c, J, Jc, dI[e] / d2, dJc, &dE[e], &dEp[e]);
        }
        /* 3. per-wire KKT tangent */
        #pragma omp parallel for schedule(dynamic, 4)
        for (long w = 0; w < Nw; ++w) {
            const int n = s->wn[w];
            const int ci = s->wcoil[w];
            const double ddIt = (dramp ? dramp[ci] : 0.0) * dt;
            const long *el = s->welem + s->wire_off[w];
            double *A = dalloc((long)n * n), *x = dalloc(n), *y = dalloc(n);
            memcpy(A, s->Mww[w], sizeof(double) * (size_t)n * n);
            for (int i = 0; i < n; ++i) {
                const long e = el[i];
                const double d2 = s->d[e] * s->d[e];
                const double kap = 2.0 * ORC_PI * s->r[e] / d2;
                A[i * n + i] += dt * kap * s->Ep[e];
                x[i] = -ddIt * s->psi[e] - dt * 2.0 * ORC_PI * s->r[e] * dE[e]
                       - dt * kap * dEp[e] * s->dI[e];
                y[i] = 1.0;
            }
            if (cholesky(A, n) == 0) {
                chol_solve(A, n, x);
                chol_solve(A, n, y);
                double sx = 0.0, sy = 0.0;
                for (int i = 0; i < n; ++i) { sx += x[i]; sy += y[i]; }
                const double dmu = (sx - ddIt) / sy;
                for (int i = 0; i < n; ++i) ddI[el[i]] = x[i] - dmu * y[i];
            }
            free(A); free(x); free(y);
        }
        /* 4. current and Joule-source tangents */
        nsum qs = {0.0, 0.0};
        for (long e = 0; e < N; ++e) {
            const double d2 = s->d[e] * s->d[e];
            const double I1 = s->I[e];
            dI[e] += ddI[e];
            const double Elin = s->E[e] + s->Ep[e] * s->dI[e] / d2;
            const double dElin = dE[e] + dEp[e] * s->dI[e] / d2 + s->Ep[e] * ddI[e] / d2;
            dq[e] = dElin * (I1 / d2) + Elin * (dI[e] / d2);
            ns_add(&qs, dt * s->V[e] * dq[e]);
        }
        dQ += ns_val(&qs);
        /* 5. heat tangent, re-deriving the primal substeps from u^k */
        memcpy(usub, uk, sizeof(double) * (size_t)N);
        memcpy(Tsub, Tk, sizeof(double) * (size_t)N);
        for (int sub = 0; sub < s->n_sub; ++sub) {
            for (long e = 0; e < N; ++e)
                dTsub[e] = du[e] / (c->C0 * pow(Tsub[e] / c->T_ref, c->cp_exp));
            for (long e = 0; e < N; ++e) {
                double flux = s->Gb[e] * (c->T_bath - Tsub[e]);
                double dflux = -s->Gb[e] * dTsub[e];
                for (int f = 0; f < 4; ++f) {
                    const long nbr = s->nb[4 * e + f];
                    if (nbr >= 0) {
                        flux += s->G[4 * e + f] * (Tsub[nbr] - Tsub[e]);
                        dflux += s->G[4 * e + f] * (dTsub[nbr] - dTsub[e]);
                    }
                }
                unew[e] = usub[e] + hs / s->V[e] * flux + hs * s->q[e];
                dunew[e] = du[e] + hs / s->V[e] * dflux + hs * dq[e];
            }
            for (long e = 0; e < N; ++e) {
                usub[e] = unew[e];
                Tsub[e] = T_of_u(c, unew[e]);
                du[e] = dunew[e];
            }
        }
        /* 6. peak temperature raised in this step */
        if (s->Tpeak_k == s->step && s->Tpeak_e >= 0) {
            const long e = s->Tpeak_e;
            dTpeak = du[e] / (c->C0 * pow(s->T[e] / c->T_ref, c->cp_exp));
        }
    }
    if (obj) { obj[0] = s->Q; obj[1] = s->Tpeak; }
    if (dobj) { dobj[0] = dQ; dobj[1] = dTpeak; }
    void *p[] = {dI, du, Ik, Tk, uk, dBr, dBz, dE, dEp, ddI, dq, Tsub, usub, dTsub, unew, dunew};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(p[i]);
    orc_destroy(s);
    return rc;
}
