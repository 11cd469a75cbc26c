// coil_kernels.hip -- gfx950 kernels of the coil quench time step.
//
// Field pass (the O(N^2) part; paper, Methods "Numerical Algorithm": the field
// of every subelement is updated from the net currents of all subelements):
//   B_e = sum_{j != e} G_B(e, j) I_j over the elements of the same coil, with
//   the coaxial-ring Green's function
//     B_z = mu0 I / (2 pi al2 be) [ (a^2 - r^2 - dz^2) E + al2 K ]
//     B_r = mu0 I dz / (2 pi r al2 be) [ (a^2 + r^2 + dz^2) E - al2 K ]
//   al2 = (r-a)^2 + dz^2, be2 = (r+a)^2 + dz^2, m1 = 1 - k^2 = al2 / be2,
//   K, E the complete elliptic integrals (polynomial-log forms, on the fly).
// Coordinates are grid indices inside the coil (r = (rho0 + i_r + 1/2) d,
// z = (i_z + 1/2) d + z0): r - a and dz are exact small integers in FP32 as in
// FP64, so al2 is exact and the near-singular argument m1 carries one rounding.
//
// Tiling: a workgroup of 64..256 threads owns as many targets (one per thread);
// sources stream through LDS in stages of 256 and are read as wave-wide
// broadcasts.  Work items (target block x source chunk) write partial sums to
// part[chunk][target]; the consumer reduces them in a fixed order.
// Mixed precision: per (64-target group, 64-source group) pair the bounding
// boxes bound m1 from below; pairs that may reach m1 < m1_near (k > near_k)
// run entirely in FP64, the others in FP32 with one plain FP32 partial per
// 64-source group and Kahan compensation across groups.  The branch is uniform
// per wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "coil_internal.h"
#include "coil_device.h"

namespace coilq {

// ------------------------------------------------------------------ field pass
template <int MIXED>
__global__ __launch_bounds__(256) void k_field(DevState s, RunConst rc) {
    __shared__ float4 sp[kStage];  // (i_r, i_z, strength fp32, 0)
    __shared__ double ss[kStage];  // strength fp64
    const int tid = threadIdx.x;
    for (int it = blockIdx.x; it < s.nitems; it += gridDim.x) {
        const PairItem item = s.items[it];
        const CoilDev c = s.coils[item.coil];
        const int t = item.t0 + tid;
        const bool tact = tid < item.tn;
        const float2 tp = s.gpos[tact ? t : item.t0];
        const double tr = tp.x, tz = tp.y;
        const double c2t = c.c2d + tr;
        const float tr32 = tp.x, tz32 = tp.y;
        const float c2t32 = c.c2f + tp.x;
        // this wavefront's target group (t0 is group aligned)
        const int wbase = item.t0 + (tid & ~63);
        const bool wact = wbase < item.t0 + item.tn;
        int4 tb = make_int4(0, 0, 0, 0);
        if (MIXED && wact) tb = s.bbox[c.group_off + (wbase - c.off) / kGroup];
        double nr = 0.0, nz = 0.0;
        float fr = 0.f, fz = 0.f, cr = 0.f, cz = 0.f;
        const int send = item.s0 + item.sn;
        for (int s0 = item.s0; s0 < send; s0 += kStage) {
            const int cnt = min(kStage, send - s0);
            __syncthreads();
            for (int i = tid; i < cnt; i += blockDim.x) {
                const float2 p = s.gpos[s0 + i];
                const double sv = s.I[s0 + i] * c.kscale;
                sp[i] = make_float4(p.x, p.y, (float)sv, 0.f);
                ss[i] = sv;
            }
            __syncthreads();
            if (!wact) continue;
            for (int g0 = 0; g0 < cnt; g0 += kGroup) {
                const int gn = min(kGroup, cnt - g0);
                bool near = true;
                if (MIXED) {
                    const int4 sb = s.bbox[c.group_off + (s0 + g0 - c.off) / kGroup];
                    near = groups_near(tb, sb, c.c2f, rc.m1_near);
                }
                if (near) {
#pragma unroll 4
                    for (int j = g0; j < g0 + gn; ++j) {
                        const float4 q = sp[j];
                        pair64(tr - (double)q.x, tz - (double)q.y, c2t + (double)q.x, ss[j], nr, nz);
                    }
                } else {
                    float pr = 0.f, pz = 0.f;
#pragma unroll 8
                    for (int j = g0; j < g0 + gn; ++j) {
                        const float4 q = sp[j];
                        pair32(tr32 - q.x, tz32 - q.y, c2t32 + q.x, q.z, pr, pz);
                    }
                    kahan_add(fr, cr, pr);
                    kahan_add(fz, cz, pz);
                }
            }
        }
        if (tact) {
            const double br = nr + ((double)fr - (double)cr);
            const double bz = nz + ((double)fz - (double)cz);
            s.part[(size_t)item.chunk * s.N + t] = make_double2(br, bz);
        }
    }
}

// B at element e from the partial sums (FP64, fixed order)
__device__ __forceinline__ void field_at(const DevState &s, const CoilDev &c, int e, double Ba,
                                         double &br, double &bz) {
    double xr = 0.0, xz = 0.0;
    const int nk = field_slots(s, c);
    // the slots are summed in order; their loads are issued 16 at a time so
    // that they are in flight together
    int k = 0;
    for (; k + 16 <= nk; k += 16) {
        double2 p[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) p[q] = s.part[(size_t)(k + q) * s.N + e];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            xr += p[q].x;
            xz += p[q].y;
        }
    }
    for (; k < nk; ++k) {
        const double2 p = s.part[(size_t)k * s.N + e];
        xr += p.x;
        xz += p.y;
    }
    br = xr / s.rho[e];
    bz = xz + Ba;
}

__global__ __launch_bounds__(256) void k_field_finalize(DevState s, RunConst rc, const int *elem_coil) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.N) return;
    const CoilDev c = s.coils[elem_coil[e]];
    const double Ba = rc.dBa_dt * (double)s.sc->step * rc.dt;
    double br, bz;
    field_at(s, c, e, Ba, br, bz);
    s.Br[e] = br;
    s.Bz[e] = bz;
}

// Per-wire bookkeeping of a step, after its solve: Q_w, U_w, max |J|/Jc, the
// status bits, the flux-jump onset (|J/Jc| > 1) and the quench criterion (the
// wire's resistivity sum V E J / sum V J^2 of this step's local law against
// 0.95 rho_n).  J0 = J^k of the lane's element; lane 0 of the wire's
// wavefront writes (a workgroup may hold several wires).
__device__ __forceinline__ void wire_diagnostics(const DevState &s, const RunConst &rc, int w, int e, bool act,
                                                 double J0, const Local &lo, unsigned bad, double qv, double U,
                                                 bool clear_flag) {
    const double qw = wave_sum(act ? rc.dt * s.V[e] * qv : 0.0);
    const double mx = wave_max(lo.x);
    bad = wave_or(bad);
    double sEJ = 0.0, sJJ = 0.0, sV = 0.0, Tw = 0.0;
    if (rc.rho_n > 0.0) {
        const double Ve = act ? s.V[e] : 0.0;
        sEJ = wave_sum(Ve * lo.E * J0);
        sJJ = wave_sum(Ve * J0 * J0);
        sV = wave_sum(Ve);
        Tw = wave_max(act ? s.T[0][e] : -INFINITY);
    }
    if ((threadIdx.x & 63) == 0) {
        const double Qold = s.Qw[w];
        if (!s.cg_defer) {
            s.Uw[w] = U;
            s.wq[w] = qw;
            s.Qw[w] = Qold + qw;
        }
        s.wmaxx[w] = mx;
        if (clear_flag) s.wflag[w] = 0;
        if (bad) atomicOr(&s.sc->status, bad);
        // flux-jump onset and quench of the wire at step k
        const double kstep = (double)s.sc->step;
        if (s.onset[w] < 0.0 && mx > 1.0) {
            s.onset[w] = kstep;
            s.Qon[w] = Qold;
        }
        if (rc.rho_n > 0.0 && s.quench[w] < 0.0 && sJJ > 0.0 && sEJ / sJJ > 0.95 * rc.rho_n) {
            s.quench[w] = kstep;
            s.Qqu[w] = Qold;
            s.Tqu[w] = Tw;
            s.Pqu[w] = sEJ / sV;
        }
    }
}

// One linearised implicit Euler step of length h for the wire, from the local
// law lo of the lane's element (E, E' at the step's currents):
//   (M_ww + h diag(2 pi r E'/d^2)) dI + h U 1 = b,  1^T dI = ramp h,
//   b = -ramp h Psi_u - pi r^2 dBa/dt h - h 2 pi r E,
// A factorised in LDS.  dIt_h = ramp h, dBa_h = dBa/dt h.
__device__ unsigned be_step_lds(double *sm, const double *M, int n, int lane, bool act, double h,
                                const Local &lo, double re, double d2, double psi, double dIt_h, double dBa_h,
                                double &dI, double &U) {
    __syncthreads();  // the previous factor's last reads
    load_wire_matrix(sm, M, n, lane, act, h * 2.0 * kPi * re * lo.Ep / d2);
    unsigned bad = chol_lds(sm, n, lane, act, sm + packed_size(n));
    double xv = act ? -dIt_h * psi - kPi * re * re * dBa_h - h * 2.0 * kPi * re * lo.E : 0.0;
    double yv = act ? 1.0 : 0.0;
    solve2_lds(sm, n, lane, act, xv, yv);
    const double sx = wave_sum(act ? xv : 0.0);
    const double sy = wave_sum(act ? yv : 0.0);
    U = (sx - dIt_h) / (h * sy);
    dI = act ? xv - h * U * yv : 0.0;
    return bad;
}

// Variable-step integration of the wire's currents over the step, with B^k
// and T^k (so Jc) held: substeps h = dt / 2^m; an attempt takes one step of h
// and two of h/2 (the local law re-evaluated at the midpoint currents); with
// I1, I2 their results, err = max_e |I2 - I1| / (em_tol max(|I2|, Jc d^2)).
// err <= 1 keeps 2 I2 - I1 (local extrapolation) and advances; otherwise m
// grows by one and the attempt is repeated (kept at the finest level).  After
// a kept substep with err <= 1/4 at a multiple of 2h, m falls by one.  Every
// step starts at m = 0.  The Joule source of the half steps, E_lin J^{new},
// is accumulated times their length; the loop voltage as 2 U2 - U1; the flux
// as 2 (dPhi_a + dPhi_b) - dPhi_1, each dPhi = -h (2 pi r E_lin + U) from its
// own circuit equation.  Returns dI, the step's mean q and U, and the flux
// change; every exit condition is wave-uniform.
__device__ unsigned em_integrate(double *sm, const DevState &s, const RunConst &rc, const CoilDev &c,
                                 const double *M, int n, int lane, bool act, int w, int e, double I0,
                                 double br, double bz, double &dI, double &qv, double &U, double &dPhi, int &nsub) {
    const double dt = rc.dt, d2 = c.d * c.d, re = act ? s.r[e] : 0.0, psi = act ? s.psi[e] : 0.0;
    const double cw = s.cw[w], jcs = act ? s.jcs[e] : 0.0, T = act ? s.T[0][e] : rc.T_bath;
    const int L = rc.em_levels;
    const long long full = 1LL << L;
    long long pos = 0;
    int m = 0;
    unsigned bad = 0;
    double Iv = act ? I0 : 0.0, qa = 0.0, Ua = 0.0, ph = 0.0;
    nsub = 0;
    while (pos < full) {
        const double h = ldexp(dt, -m), hh = 0.5 * h;
        const double dIt_h = ldexp(c.dIt, -m), dBa_h = ldexp(rc.dBa_dt * dt, -m);
        Local la, lm;
        bad |= act ? local_law(rc, cw, jcs, Iv / d2, T, br, bz, la) : 0u;
        if (!act) la.E = la.Ep = la.Jc = 0.0;
        double d1, U1, da, Uh1, db, Uh2;
        bad |= be_step_lds(sm, M, n, lane, act, h, la, re, d2, psi, dIt_h, dBa_h, d1, U1);
        bad |= be_step_lds(sm, M, n, lane, act, hh, la, re, d2, psi, 0.5 * dIt_h, 0.5 * dBa_h, da, Uh1);
        const double Im = Iv + da;
        bad |= act ? local_law(rc, cw, jcs, Im / d2, T, br, bz, lm) : 0u;
        if (!act) lm.E = lm.Ep = 0.0;
        bad |= be_step_lds(sm, M, n, lane, act, hh, lm, re, d2, psi, 0.5 * dIt_h, 0.5 * dBa_h, db, Uh2);
        const double I2 = Im + db, I1 = Iv + d1;
        const double sc = rc.em_tol * fmax(fabs(I2), la.Jc > 0.0 ? la.Jc * d2 : 0.0);
        const double dif = fabs(I2 - I1);
        const double ei = !act ? 0.0 : (sc > 0.0 ? dif / sc : (dif == 0.0 ? 0.0 : INFINITY));
        const double err = wave_max(ei);
        if (err > 1.0 && m < L) {
            ++m;
            continue;
        }
        const double Ea = la.E + la.Ep * da / d2, Eb = lm.E + lm.Ep * db / d2, E1 = la.E + la.Ep * d1 / d2;
        qa += hh * (Ea * (Im / d2) + Eb * (I2 / d2));
        ph += 2.0 * (-hh * (2.0 * kPi * re * Ea + Uh1) - hh * (2.0 * kPi * re * Eb + Uh2)) +
              h * (2.0 * kPi * re * E1 + U1);
        Ua += h * (Uh1 + Uh2 - U1);
        Iv = 2.0 * I2 - I1;
        pos += 1LL << (L - m);
        ++nsub;
        if (err <= 0.25 && m > 0 && pos % (1LL << (L - m + 1)) == 0) --m;
    }
    dI = act ? Iv - I0 : 0.0;
    qv = qa / dt;
    U = Ua / dt;
    dPhi = ph;
    return bad;
}

// ------------------------------------------------------------------ local law + per-wire A-V solve
// One wavefront per wire, one element per lane (n_e <= 64).  The wire matrix is
// A = M_ww + dt diag(2 pi r E'/d^2).  Two kernels per step:
//   k_wire<1>: workgroups of kFastWires wavefronts, all wires of one layer,
//     which share the layer's precomputed inverse staged once in LDS.  When
//     every diagonal addition leaves M_ee unchanged in FP64, A equals the
//     layer's inductance block bitwise and the solution uses that inverse
//     (x = M^-1 b, y = M^-1 1); otherwise the wire is flagged and left
//     untouched;
//   k_wire<0>: flagged wires only; A in LDS (packed lower triangle by
//     columns), right-looking Cholesky and two triangular solves.
// Optional recording (adjoint recompute): I^k, B^k and dI of the step; optional
// field source (adjoint recompute from a stored field history).
template <int FAST>
__global__ __launch_bounds__(FAST ? 64 * kFastWires : 64) void k_wire(DevState s, RunConst rc) {
    extern __shared__ double sm[];
    const int lane = threadIdx.x & 63;
    int w;
    bool live = true;
    CoilDev c;
    if (FAST) {
        // four wires of one layer (so of one coil): every wave of the
        // workgroup reaches the barrier that stages the layer inverse below
        const int w0 = s.fast_w0[blockIdx.x];
        c = s.coils[s.wire_coil[w0]];
        const int v = threadIdx.x >> 6;
        live = v < c.turns - (w0 - c.wire_off) % c.turns;  // past the layer's last wire: no wire
        w = live ? w0 + v : w0;
    } else {
        w = blockIdx.x;
        if (s.wflag[w] == 0) return;
        c = s.coils[s.wire_coil[w]];
    }
    const int lw = w - c.wire_off;
    const int layer = lw / c.turns;
    const int n = c.ne2;
    const bool act = lane < n;
    const int e = c.off + lw * n + (act ? lane : 0);
    const double dt = rc.dt;
    const double tk = (double)s.sc->step * dt;
    const double dBa = rc.dBa_dt * dt;

    // the element's loads and its local law are issued before the fast
    // path stages the layer inverse, so that their latencies overlap
    const size_t lay = (size_t)(c.layer_off + layer);
    double br, bz;
    if (s.src_Br) {
        br = s.src_Br[e];
        bz = s.src_Bz[e];
    } else {
        field_at(s, c, e, rc.dBa_dt * tk, br, bz);
    }
    const double I0 = s.I[e];
    const double d2 = c.d * c.d;
    Local lo;
    unsigned bad = act ? local_law(rc, s.cw[w], s.jcs[e], I0 / d2, s.T[0][e], br, bz, lo) : 0u;
    if (!act) { lo.E = lo.Ep = lo.x = lo.Jc = lo.p = 0.0; }
    const double re = s.r[e];
    const double *M = s.Mlay + lay * n * n;
    const double diag_add = dt * 2.0 * kPi * re * lo.Ep / d2;
    const double b = act ? (-c.dIt * s.psi[e] - kPi * re * re * dBa - dt * 2.0 * kPi * re * lo.E) : 0.0;
    double mee = 1.0, ylv = 0.0, sylv = 0.0;
    if (FAST) {
        mee = act ? M[(size_t)lane * n + lane] : 1.0;
        ylv = act ? s.yl[lay * n + lane] : 0.0;
        sylv = s.syl[lay];
        // the layer inverse into LDS, eight values per thread at a time with
        // their loads issued at once (a loop that stores each value as it
        // arrives pays the memory latency once per value: 16 times at n_e = 64);
        // loads past the end re-read the last.  Issued before the local law
        // instead, they held registers across it (98-107 VGPRs against 79:
        // four waves per SIMD instead of six), which slowed the wire phase of
        // the 17,152-wire ensemble from 60 to 70 us
        const double *Mi = s.Minv + lay * n * n;
        constexpr int kStage = 8, kStep = 64 * kFastWires;
        const int nn = n * n;
        for (int b = 0; b < nn; b += kStage * kStep) {
            double mv[kStage];
#pragma unroll
            for (int k = 0; k < kStage; ++k) mv[k] = Mi[min(b + (int)threadIdx.x + k * kStep, nn - 1)];
#pragma unroll
            for (int k = 0; k < kStage; ++k) {
                const int i = b + (int)threadIdx.x + k * kStep;
                if (i < nn) sm[i] = mv[k];
            }
        }
        __syncthreads();
        if (!live) return;
    }
    double xv, yv, sy;
    if (FAST) {
        const int same = act ? (mee + diag_add == mee) : 1;
        if (!__all(same)) {
            if (lane == 0) s.wflag[w] = 1;
            return;
        }
        if (s.emsub && lane == 0) s.emsub[w] = 1.0;  // a linear step: one substep is exact
        xv = matvec_lds(sm, n, act, lane, b);
        yv = ylv;
        sy = sylv;
    } else {
        load_wire_matrix(sm, M, n, lane, act, diag_add);
        bad |= chol_lds(sm, n, lane, act, sm + packed_size(n));
        if (s.cg_defer) {  // the factor, for the coupled solve's preconditioner (every lane copies)
            double *L = s.cg_L + (size_t)w * packed_size(s.max_ne2);
            for (int i = lane; i < packed_size(n); i += 64) L[i] = sm[i];
        }
        xv = b;
        yv = act ? 1.0 : 0.0;
        solve2_lds(sm, n, lane, act, xv, yv);
        sy = wave_sum(act ? yv : 0.0);
    }
    const double sx = wave_sum(act ? xv : 0.0);
    const double U = (sx - c.dIt) / (dt * sy);
    const double dI = act ? xv - dt * U * yv : 0.0;
    double qv = 0.0;
    if (s.cg_defer) {
        // coupled solve: dI is its starting point; the step's updates of I, q,
        // Phi, U_w and Q_w follow once it has converged
        if (act) {
            s.dI[e] = dI;
            s.E[e] = lo.E;
            s.Ep[e] = lo.Ep;
            s.Jc[e] = lo.Jc;
            s.Br[e] = br;
            s.Bz[e] = bz;
            if (s.rec_I) s.rec_I[e] = I0;
            if (s.rec_Br) {
                s.rec_Br[e] = br;
                s.rec_Bz[e] = bz;
            }
        }
    } else if (act) {
        const double I1 = I0 + dI;
        const double Elin = lo.E + lo.Ep * dI / d2;
        qv = Elin * (I1 / d2);
        // flux update Phi += M_ww dI + dI_t Psi_u + pi r^2 dB_a.  The solved
        // system A dI = b - dt U 1 (A = M_ww in the fast path, M_ww plus the
        // diagonal otherwise) gives M_ww dI = b - dt U - (A - M_ww) dI, so the
        // update is the circuit equation itself, without a second product:
        // -dt (2 pi r E + U), with E linearised at I + dI when the diagonal
        // entered the solve.
        s.Phi[e] += -dt * (2.0 * kPi * re * (FAST ? lo.E : Elin) + U);
        s.I[e] = I1;
        s.dI[e] = dI;
        s.E[e] = lo.E;
        s.Ep[e] = lo.Ep;
        s.q[e] = qv;
        s.Jc[e] = lo.Jc;
        s.Br[e] = br;
        s.Bz[e] = bz;
        if (s.rec_I) s.rec_I[e] = I0;
        if (s.rec_Br) {
            s.rec_Br[e] = br;
            s.rec_Bz[e] = bz;
        }
        if (s.rec_dI) s.rec_dI[e] = dI;
        if (!isfinite(I1) || !isfinite(qv)) bad |= ST_NONFINITE;
    }
    wire_diagnostics(s, rc, w, e, act, I0 / (c.d * c.d), lo, bad, qv, U, !FAST);
}

// Variable-step wires: those the fast path flagged, with em_tol > 0 (in place
// of k_wire<0>; transport coupling only, so no deferred solve; no adjoint, so
// no recording).
__global__ __launch_bounds__(64) void k_wire_em(DevState s, RunConst rc) {
    extern __shared__ double sm[];
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    if (s.wflag[w] == 0) return;
    const CoilDev c = s.coils[s.wire_coil[w]];
    const int lw = w - c.wire_off;
    const int n = c.ne2;
    const bool act = lane < n;
    const int e = c.off + lw * n + (act ? lane : 0);
    const double tk = (double)s.sc->step * rc.dt;
    double br, bz;
    field_at(s, c, e, rc.dBa_dt * tk, br, bz);
    const double I0 = s.I[e];
    const double d2 = c.d * c.d;
    Local lo;
    unsigned bad = act ? local_law(rc, s.cw[w], s.jcs[e], I0 / d2, s.T[0][e], br, bz, lo) : 0u;
    if (!act) { lo.E = lo.Ep = lo.x = lo.Jc = lo.p = 0.0; }
    const double *M = s.Mlay + (size_t)(c.layer_off + lw / c.turns) * n * n;
    double dI, qv, U, dPhi;
    int nsub;
    bad |= em_integrate(sm, s, rc, c, M, n, lane, act, w, e, I0, br, bz, dI, qv, U, dPhi, nsub);
    if (act) {
        const double I1 = I0 + dI;
        s.Phi[e] += dPhi;
        s.I[e] = I1;
        s.dI[e] = dI;
        s.E[e] = lo.E;
        s.Ep[e] = lo.Ep;
        s.q[e] = qv;
        s.Jc[e] = lo.Jc;
        s.Br[e] = br;
        s.Bz[e] = bz;
        if (!isfinite(I1) || !isfinite(qv)) bad |= ST_NONFINITE;
    }
    if (lane == 0) s.emsub[w] = (double)nsub;
    wire_diagnostics(s, rc, w, e, act, I0 / d2, lo, bad, act ? qv : 0.0, U, true);
}

// ------------------------------------------------------------------ subelement model
// The wire's ne x ne elements form sq x sq square subelements of sb x sb
// elements (sb = ne / sq); element (a, b) of the wire (lane a ne + b) belongs
// to subelement (a / sb) sq + b / sb.  Sum over the elements of subelement t of
// a vector staged in LDS, in ascending element order.
__device__ __forceinline__ double subelement_sum(const double *v, int t, int sq, int sb, int ne) {
    const int a0 = (t / sq) * sb, b0 = (t % sq) * sb;
    double acc = 0.0;
    for (int a = 0; a < sb; ++a)
        for (int b = 0; b < sb; ++b) acc += v[(a0 + a) * ne + b0 + b];
    return acc;
}

// One wavefront per wire, one element per lane.  The element current is
// I_H + I_I: the field-driven part keeps zero net current in every subelement,
// the transport part carries the wire's transport current; both respond
// through A = M_ww + dt diag(2 pi r E'/d^2), driven by the resistivity
// rho = E/J of the total J^k (E' where J = 0) times their own current density:
//   A dI_H = b_H - P (dt U_s),  P^T dI_H = 0     (one voltage per subelement)
//   A dI_I = b_I - dt U_I 1,    1^T dI_I = dI_t  (one voltage per wire)
//   b_H = -dI_t Psi_u - pi r^2 dB_a - dt 2 pi r rho J_H,  b_I = -dt 2 pi r rho J_I
// with P the element-to-subelement incidence.  A is factorised in LDS; the
// subelement voltages solve S (dt U_s) = P^T A^-1 b_H with S = P^T A^-1 P
// (ns x ns, built from ns solves, four at a time, and factorised in LDS), and
// dI_H = A^-1 b_H - A^-1 P (dt U_s).  The wire's voltage is the element mean of
// the loop voltages, U_I + mean_s U_s.  LDS: A and S as packed lower triangles,
// each followed by its factorisation's store sink, and four staging columns
// of n.
__global__ __launch_bounds__(64) void k_wire_sub(DevState s, RunConst rc) {
    extern __shared__ double sm[];
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const CoilDev c = s.coils[s.wire_coil[w]];
    const int lw = w - c.wire_off;
    const int layer = lw / c.turns;
    const int n = c.ne2;
    const int sq = s.nsubel, ns = sq * sq, sb = c.ne / sq;
    double *Lr = sm + packed_size(n) + kCholPad;  // the factor by rows (backward sweeps)
    double *S = Lr + packed_size(n);
    double *col = S + packed_size(ns) + kCholPad;
    const bool act = lane < n;
    const bool sact = lane < ns;
    const int e = c.off + lw * n + (act ? lane : 0);
    const int sub = act ? ((lane / c.ne) / sb) * sq + (lane % c.ne) / sb : 0;
    const double dt = rc.dt;
    const double tk = (double)s.sc->step * dt;
    const double dBa = rc.dBa_dt * dt;
    double br, bz;
    field_at(s, c, e, rc.dBa_dt * tk, br, bz);
    const double I0 = s.I[e], IH0 = s.IH[e];
    const double d2 = c.d * c.d;
    Local lo;
    unsigned bad = act ? local_law(rc, s.cw[w], s.jcs[e], I0 / d2, s.T[0][e], br, bz, lo) : 0u;
    if (!act) { lo.E = lo.Ep = lo.x = lo.Jc = lo.p = 0.0; }
    const double re = s.r[e];
    const double J = I0 / d2, JH = IH0 / d2;
    const double rho = (J != 0.0) ? lo.E / J : lo.Ep;
    load_wire_matrix(sm, s.Mlay + (size_t)(c.layer_off + layer) * n * n, n, lane, act,
                     dt * 2.0 * kPi * re * lo.Ep / d2);
    bad |= chol_lds(sm, n, lane, act, sm + packed_size(n));
    factor_rows_lds(sm, Lr, n, lane, act);
    double v3[3];
    v3[0] = act ? -c.dIt * s.psi[e] - kPi * re * re * dBa - dt * 2.0 * kPi * re * rho * JH : 0.0;
    v3[1] = act ? -dt * 2.0 * kPi * re * rho * (J - JH) : 0.0;
    v3[2] = act ? 1.0 : 0.0;
    solve_lds_rows<3>(sm, Lr, n, lane, act, v3);
    const double xh = v3[0], xi = v3[1], yv = v3[2];
    // S = P^T A^-1 P, column v = the subelement sums of A^-1 p_v
    for (int v0 = 0; v0 < ns; v0 += 4) {
        double y4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) y4[q] = (act && sub == v0 + q) ? 1.0 : 0.0;
        solve_lds_rows<4>(sm, Lr, n, lane, act, y4);
        __syncthreads();
        if (act)
#pragma unroll
            for (int q = 0; q < 4; ++q) col[q * n + lane] = y4[q];
        __syncthreads();
        if (sact)  // the lower triangle of S: rows lane >= column v0 + q
            for (int q = 0; q < 4 && v0 + q < ns; ++q)
                if (lane >= v0 + q) S[pcol(ns, v0 + q) + lane - (v0 + q)] = subelement_sum(col + q * n, lane, sq, sb, c.ne);
    }
    __syncthreads();
    if (act) col[lane] = xh;
    __syncthreads();
    double u1[1] = {sact ? subelement_sum(col, lane, sq, sb, c.ne) : 0.0};
    bad |= chol_lds(S, ns, lane, sact, S + packed_size(ns));
    solve_lds<1>(S, ns, lane, sact, u1);     // dt U_s of subelement `lane`
    const double pu = __shfl(u1[0], sub);         // ... of this lane's subelement
    const double usum = wave_sum(sact ? u1[0] : 0.0);
    double z1[1] = {act ? pu : 0.0};
    solve_lds_rows<1>(sm, Lr, n, lane, act, z1);
    const double dIH = act ? xh - z1[0] : 0.0;
    const double sx = wave_sum(act ? xi : 0.0);
    const double sy = wave_sum(act ? yv : 0.0);
    const double UI = (sx - c.dIt) / (dt * sy);
    const double dI = act ? dIH + (xi - dt * UI * yv) : 0.0;
    double qv = 0.0;
    if (act) {
        const double I1 = I0 + dI;
        const double Elin = lo.E + lo.Ep * dI / d2;
        qv = Elin * (I1 / d2);
        // Phi += M_ww dI + dI_t Psi_u + pi r^2 dB_a, from the circuit equation
        // of the two solves together (rho J = E)
        s.Phi[e] += -dt * (2.0 * kPi * re * Elin + UI) - pu;
        s.I[e] = I1;
        s.IH[e] = IH0 + dIH;
        s.dI[e] = dI;
        s.E[e] = lo.E;
        s.Ep[e] = lo.Ep;
        s.q[e] = qv;
        s.Jc[e] = lo.Jc;
        s.Br[e] = br;
        s.Bz[e] = bz;
        if (!isfinite(I1) || !isfinite(qv)) bad |= ST_NONFINITE;
    }
    wire_diagnostics(s, rc, w, e, act, J, lo, bad, qv, UI + usum / ((double)ns * dt), false);
}

// ------------------------------------------------------------------ heat
// Tiled explicit substeps.  A workgroup owns a kHT x kHT tile of a coil's
// (r, z) grid and loads it with a halo of H cells (u, T of the source buffer,
// q) into LDS; substep k (0 <= k < H) updates the cells at least k + 1 cells
// inside the loaded region, whose neighbours were all updated by substep
// k - 1, so after H substeps the owned tile is exact.  Neighbours and face
// conductances follow from the grid indices and a per-row table (the same
// host-computed values as the per-element conductances, summed in the same
// face order), so no per-element geometry is read.  Per substep the owned
// cells' border outflow is summed per tile; the last substep of a step also
// keeps the tile's largest T and its lowest public index.
__device__ __forceinline__ int elem_of(const CoilDev &c, int ir, int iz) {
    return c.off + ((ir / c.ne) * c.turns + iz / c.ne) * c.ne2 + (ir % c.ne) * c.ne + iz % c.ne;
}

__global__ __launch_bounds__(256) void k_heat_tile(DevState s, RunConst rc, int src, int dst, int sub0, int H,
                                                   int last) {
    extern __shared__ double sh[];
    __shared__ double red_o[2][4];  // per substep parity: written before the next read
    __shared__ double red_t[4];
    __shared__ long long red_i[4];
    const int Wd = kHT + 2 * H, ncell = Wd * Wd;
    double *Ta = sh, *Tb = sh + ncell, *ul = sh + 2 * ncell, *ql = sh + 3 * ncell;
    HeatRow *rows = reinterpret_cast<HeatRow *>(sh + 4 * ncell);
    const int tid = threadIdx.x;
    // the tile's coil: the last coil whose first tile is <= blockIdx.x
    int lo = 0, hi = s.ncoils - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (s.coils[mid].tile_off <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const CoilDev c = s.coils[lo];
    const int lt = (int)blockIdx.x - c.tile_off;
    const int nr = c.layers * c.ne, nz = c.turns * c.ne;
    const int ir0 = (lt / c.ntile_z) * kHT - H, iz0 = (lt % c.ntile_z) * kHT - H;
    const double *Tsrc = s.T[src], *usrc = s.u[src];
    for (int k = tid; k < ncell; k += 256) {
        const int ir = ir0 + k / Wd, iz = iz0 + k % Wd;
        if (ir >= 0 && ir < nr && iz >= 0 && iz < nz) {
            const int e = elem_of(c, ir, iz);
            Ta[k] = Tsrc[e];
            ul[k] = usrc[e];
            ql[k] = s.q[e];
        }
    }
    for (int i = tid; i < Wd; i += 256) {
        const int ir = ir0 + i;
        if (ir >= 0 && ir < nr) rows[i] = s.hrow[c.row_off + ir];
    }
    __syncthreads();
    const double hs = rc.dt / (double)s.nsub;
    double *Tc = Ta, *Tn = Tb;
    for (int k = 0; k < H; ++k) {
        const int sub = sub0 + k;
        const int a = k + 1, wr = Wd - 2 * (k + 1);
        double outv = 0.0;
        for (int m = tid; m < wr * wr; m += 256) {
            const int i = a + m / wr, j = a + m % wr;
            const int ir = ir0 + i, iz = iz0 + j;
            if (ir < 0 || ir >= nr || iz < 0 || iz >= nz) continue;
            const int kk = i * Wd + j;
            const HeatRow R = rows[i];
            const double Te = Tc[kk];
            // border faces in the order inner, outer, lower, upper
            double gb = 0.0;
            if (ir == 0) gb += R.gbin;
            if (ir == nr - 1) gb += R.gbout;
            if (iz == 0) gb += R.gbax;
            if (iz == nz - 1) gb += R.gbax;
            double flux = gb * (rc.T_bath - Te);
            if (ir > 0) flux += R.gin * (Tc[kk - Wd] - Te);
            if (ir < nr - 1) flux += R.gout * (Tc[kk + Wd] - Te);
            if (iz > 0) flux += R.gax * (Tc[kk - 1] - Te);
            if (iz < nz - 1) flux += R.gax * (Tc[kk + 1] - Te);
            const double un = ul[kk] + hs * R.invV * flux + hs * ql[kk];
            ul[kk] = un;
            Tn[kk] = T_of_u(rc, un);
            if (i >= H && i < H + kHT && j >= H && j < H + kHT) {  // owned cell
                outv += hs * gb * (Te - rc.T_bath);
                if (s.rec_T) s.rec_T[(size_t)sub * s.N + elem_of(c, ir, iz)] = Te;
            }
        }
        // the tile's border outflow: per wavefront (DPP sum), then the four
        // wavefronts' sums in order
        // (the barrier also orders this substep's T against the next one's reads)
        outv = wave_sum(outv);
        double *ro = red_o[k & 1];
        if ((tid & 63) == 0) ro[tid >> 6] = outv;
        __syncthreads();
        if (tid == 0) s.hb_out[(size_t)sub * s.nheat_blocks + blockIdx.x] = ((ro[0] + ro[1]) + ro[2]) + ro[3];
        double *t = Tc;
        Tc = Tn;
        Tn = t;
    }
    // owned cells out, with the tile's largest T (lowest public index on ties)
    double tm = -INFINITY;
    long long ti = LLONG_MAX;
    unsigned bad = 0u;
    for (int m = tid; m < kHT * kHT; m += 256) {
        const int i = H + m / kHT, j = H + m % kHT;
        const int ir = ir0 + i, iz = iz0 + j;
        if (ir >= nr || iz >= nz) continue;
        const int kk = i * Wd + j;
        const int e = elem_of(c, ir, iz);
        const double Tv = Tc[kk];
        s.u[dst][e] = ul[kk];
        s.T[dst][e] = Tv;
        if (!isfinite(Tv)) bad = ST_NONFINITE;
        const long long pub = (long long)c.off + (long long)ir * nz + iz;
        if (Tv > tm || (Tv == tm && pub < ti)) {
            tm = Tv;
            ti = pub;
        }
    }
    if (bad) atomicOr(&s.sc->status, bad);
    if (!last) return;
    // the tile's largest T, lowest public index on ties: per wavefront by
    // shuffles, then over the four wavefronts
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(tm, o);
        const long long yi = __shfl_xor(ti, o);
        if (y > tm || (y == tm && yi < ti)) {
            tm = y;
            ti = yi;
        }
    }
    if ((tid & 63) == 0) {
        red_t[tid >> 6] = tm;
        red_i[tid >> 6] = ti;
    }
    __syncthreads();
    if (tid == 0) {
        for (int k = 1; k < 4; ++k)
            if (red_t[k] > tm || (red_t[k] == tm && red_i[k] < ti)) {
                tm = red_t[k];
                ti = red_i[k];
            }
        s.hb_max[blockIdx.x] = tm;
        s.hb_arg[blockIdx.x] = ti;
    }
}

// ------------------------------------------------------------------ reductions
// One workgroup of kFinThreads threads: strided partial sums, then a tree.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void k_finalize(DevState s, RunConst rc) {
    __shared__ double a_q[kFinThreads], a_u[kFinThreads], a_x[kFinThreads], a_o[kFinThreads], a_t[kFinThreads];
    __shared__ long long a_i[kFinThreads];
    const int tid = threadIdx.x;
    // the running scalars are read first, so that their loads overlap the sums
    Scalars *sc = s.sc;
    double Q0 = 0.0, Qout0 = 0.0, Tpeak0 = 0.0;
    long long step0 = 0;
    if (tid == 0) {
        Q0 = sc->Q;
        Qout0 = sc->Qout;
        Tpeak0 = sc->Tpeak;
        step0 = sc->step;
    }
    double q = 0.0, u = 0.0, x = 0.0, o = 0.0, tm = -INFINITY;
    long long ti = LLONG_MAX;
#pragma unroll 4
    for (int w = tid; w < s.Nw; w += kFinThreads) {
        q += s.wq[w];
        u += s.Uw[w];
        x = fmax(x, s.wmaxx[w]);
    }
    const int no = s.hb_slots * s.nheat_blocks;
#pragma unroll 4
    for (int i = tid; i < no; i += kFinThreads) o += s.hb_out[i];
    for (int b = tid; b < s.nheat_blocks; b += kFinThreads) {
        const double v = s.hb_max[b];
        const long long iv = s.hb_arg[b];
        if (v > tm || (v == tm && iv < ti)) { tm = v; ti = iv; }
    }
    a_q[tid] = q; a_u[tid] = u; a_x[tid] = x; a_o[tid] = o; a_t[tid] = tm; a_i[tid] = ti;
    __syncthreads();
    for (int k = kFinThreads / 2; k > 0; k >>= 1) {
        if (tid < k) {
            a_q[tid] += a_q[tid + k];
            a_u[tid] += a_u[tid + k];
            a_x[tid] = fmax(a_x[tid], a_x[tid + k]);
            a_o[tid] += a_o[tid + k];
            const double v = a_t[tid + k];
            if (v > a_t[tid] || (v == a_t[tid] && a_i[tid + k] < a_i[tid])) {
                a_t[tid] = v;
                a_i[tid] = a_i[tid + k];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double Q1 = Q0 + a_q[0];
        sc->Q = Q1;
        sc->sumU = a_u[0];
        sc->maxx = a_x[0];
        sc->Qout = Qout0 + a_o[0];
        const long long stepn = step0 + 1;
        if (a_t[0] > Tpeak0) {
            sc->Tpeak = a_t[0];
            sc->Tpeak_pub = a_i[0];
            sc->Tpeak_step = stepn;
        }
        if (!isfinite(Q1)) atomicOr(&sc->status, ST_NONFINITE);
        sc->step = stepn;
    }
}

// ------------------------------------------------------------------ transport-flux pattern (init)
// Psi_u,e = sum over the other wires' elements j of M(e, j) / n_e(j), with
// Maxwell's M = mu0 be [ (1+m1)/2 K - E ] (be in metres), FP64.
__global__ __launch_bounds__(256) void k_psi(DevState s, const int *elem_coil, double *psi) {
    __shared__ float2 sp[kStage];
    const int tid = threadIdx.x;
    const int t = blockIdx.x * 256 + tid;
    const bool tact = t < s.N;
    // every element of a 256-block belongs to one coil only if coils are
    // 256-aligned; handle mixed blocks by looping over the coils it touches
    const int t_first = blockIdx.x * 256;
    const int t_last = min(s.N, t_first + 256) - 1;
    const int c_first = elem_coil[t_first], c_last = elem_coil[t_last];
    const int tc = tact ? elem_coil[t] : -1;
    double acc = 0.0;
    const float2 tp = s.gpos[tact ? t : t_first];
    for (int ci = c_first; ci <= c_last; ++ci) {
        const CoilDev c = s.coils[ci];
        const int twire = tact && tc == ci ? (t - c.off) / c.ne2 : -1;
        const double tr = tp.x, tz = tp.y;
        for (int s0 = c.off; s0 < c.off + c.n; s0 += kStage) {
            const int cnt = min(kStage, c.off + c.n - s0);
            __syncthreads();
            if (tid < cnt) sp[tid] = s.gpos[s0 + tid];
            __syncthreads();
            if (tc != ci) continue;
            for (int j = 0; j < cnt; ++j) {
                const int swire = (s0 + j - c.off) / c.ne2;
                if (swire == twire) continue;
                const float2 q = sp[j];
                const double dr = tr - (double)q.x, dz = tz - (double)q.y;
                const double sr = c.c2d + tr + (double)q.x;
                const double al2 = fma(dr, dr, dz * dz);
                const double be2 = fma(sr, sr, dz * dz);
                const double m1 = al2 / be2;
                const double L = -log(m1);
                const double K = fma(ellipk64_Q(m1), L, ellipk64_P(m1));
                const double E = fma(ellipe64_Q(m1), L, ellipe64_P(m1));
                acc += kMu0 * sqrt(be2) * c.d * (0.5 * (1.0 + m1) * K - E) / (double)c.ne2;
            }
        }
    }
    if (tact) psi[t] = acc;
}

// ------------------------------------------------------------------ field at arbitrary points
// B at probe points (r, z) from every element of every coil, FP64, physical
// coordinates (metres); B_r = 0 on the axis.  One thread per probe, sources
// staged through LDS.
__global__ __launch_bounds__(256) void k_probe(DevState s, const double *zphys, int np, const double *pr,
                                               const double *pz, double *out_br, double *out_bz) {
    __shared__ double2 sp[kStage];  // (r, z)
    __shared__ double si[kStage];   // mu0 I / (2 pi)
    const int tid = threadIdx.x;
    const int p = blockIdx.x * 256 + tid;
    const bool act = p < np;
    const double r = act ? pr[p] : 1.0, z = act ? pz[p] : 0.0;
    double ar = 0.0, az = 0.0;
    for (int s0 = 0; s0 < s.N; s0 += kStage) {
        const int cnt = min(kStage, s.N - s0);
        __syncthreads();
        if (tid < cnt) {
            sp[tid] = make_double2(s.r[s0 + tid], zphys[s0 + tid]);
            si[tid] = kMu0 / (2.0 * kPi) * s.I[s0 + tid];
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const double2 q = sp[j];
            // same pair formula in metres: dr = r - a, sr = r + a
            pair64(r - q.x, z - q.y, r + q.x, si[j], ar, az);
        }
    }
    if (act) {
        out_br[p] = r > 0.0 ? ar / r : 0.0;
        out_bz[p] = az;
    }
}

// Probes with the sources split into chunks (grid.y = chunk): partial sums
// (B_r r, B_z) of chunk c for probe p at part[c np + p]; k_probe_sum adds the
// chunks in order.  More workgroups than probes / 256 when there are few probes.
__global__ __launch_bounds__(256) void k_probe_chunk(DevState s, const double *zphys, int np, const double *pr,
                                                     const double *pz, int chunk, double2 *part) {
    __shared__ double2 sp[kStage];  // (r, z)
    __shared__ double si[kStage];   // mu0 I / (2 pi)
    const int tid = threadIdx.x;
    const int p = blockIdx.x * 256 + tid;
    const bool act = p < np;
    const double r = act ? pr[p] : 1.0, z = act ? pz[p] : 0.0;
    double ar = 0.0, az = 0.0;
    const int j0 = blockIdx.y * chunk, j1 = min(s.N, j0 + chunk);
    for (int s0 = j0; s0 < j1; s0 += kStage) {
        const int cnt = min(kStage, j1 - s0);
        __syncthreads();
        if (tid < cnt) {
            sp[tid] = make_double2(s.r[s0 + tid], zphys[s0 + tid]);
            si[tid] = kMu0 / (2.0 * kPi) * s.I[s0 + tid];
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const double2 q = sp[j];
            pair64(r - q.x, z - q.y, r + q.x, si[j], ar, az);
        }
    }
    if (act) part[(size_t)blockIdx.y * np + p] = make_double2(ar, az);
}

__global__ void k_probe_sum(int np, int nchunk, const double *pr, const double2 *part, double *out_br,
                            double *out_bz) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= np) return;
    double ar = 0.0, az = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        const double2 v = part[(size_t)c * np + p];
        ar += v.x;
        az += v.y;
    }
    const double r = pr[p];
    out_br[p] = r > 0.0 ? ar / r : 0.0;
    out_bz[p] = az;
}

// ------------------------------------------------------------------ small kernels
__global__ void k_gather(const double *src, const int *perm, int n, double *dst) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];  // internal i -> public perm[i]
}
__global__ void k_scatter(const double *src, const int *perm, int n, double *dst) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];  // public perm[i] -> internal i
}
__global__ void k_zero_int(int *p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}
__global__ void k_fill(double *p, double v, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}
// initial element currents: the coil's I0 spread evenly over each wire
__global__ void k_init_current(DevState s) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < s.N) s.I[e] = s.coils[s.elem_coil[e]].I0e;
}
__global__ void k_u_of_T(DevState s, RunConst rc) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.N) return;
    const double T = s.T[0][e];
    const double p1 = rc.cp_exp + 1.0;
    s.u[0][e] = rc.C0 * rc.T_ref / p1 * (pow(T / rc.T_ref, p1) - rc.u_a0);
}
__global__ void k_reset_scalars(Scalars *sc, double T_bath) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->Q = 0.0;
        sc->Tpeak = T_bath;
        sc->sumU = 0.0;
        sc->maxx = 0.0;
        sc->Qout = 0.0;
        sc->step = 0;
        sc->Tpeak_pub = -1;
        sc->Tpeak_step = -1;
        sc->status = 0;
        sc->pad = 0;
    }
}
__global__ __launch_bounds__(256) void k_stored(DevState s, double *out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double a = 0.0;
    for (int e = tid; e < s.N; e += 256) a += s.V[e] * s.u[0][e];
    red[tid] = a;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) *out = red[0];
}

__global__ void k_copy2(const double *a, const double *b, double *ad, double *bd, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        ad[i] = a[i];
        bd[i] = b[i];
    }
}

// ------------------------------------------------------------------ launchers
static inline int blocks_for(int n) { return (n + 255) / 256; }

hipError_t launch_field(const DevState &s, const RunConst &rc, int grid_limit, hipStream_t st) {
    if (s.nitems == 0) return hipSuccess;
    const int grid = grid_limit > 0 ? min(grid_limit, s.nitems) : s.nitems;
    if (rc.prec == COIL_MIXED)
        hipLaunchKernelGGL(k_field<1>, dim3(grid), dim3(s.tile_targets), 0, st, s, rc);
    else
        hipLaunchKernelGGL(k_field<0>, dim3(grid), dim3(s.tile_targets), 0, st, s, rc);
    return hipGetLastError();
}

hipError_t launch_field_finalize(const DevState &s, const RunConst &rc, hipStream_t st) {
    hipLaunchKernelGGL(k_field_finalize, dim3(blocks_for(s.N)), dim3(256), 0, st, s, rc, s.elem_coil);
    return hipGetLastError();
}

hipError_t launch_wire(const DevState &s, const RunConst &rc, hipStream_t st) {
    if (s.nsubel > 0) {
        const size_t ns = (size_t)s.nsubel * s.nsubel;
        const size_t lds =
            sizeof(double) * (2 * (size_t)packed_size(s.max_ne2) + kCholPad + packed_size((int)ns) + kCholPad +
                              4 * s.max_ne2);
        hipLaunchKernelGGL(k_wire_sub, dim3(s.Nw), dim3(64), lds, st, s, rc);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_wire<1>, dim3(s.nfast), dim3(64 * kFastWires), sizeof(double) * (size_t)s.max_ne2 * s.max_ne2,
                       st, s, rc);
    const size_t lds = sizeof(double) * ((size_t)packed_size(s.max_ne2) + kCholPad);
    if (rc.em_tol > 0.0)
        hipLaunchKernelGGL(k_wire_em, dim3(s.Nw), dim3(64), lds, st, s, rc);
    else
        hipLaunchKernelGGL(k_wire<0>, dim3(s.Nw), dim3(64), lds, st, s, rc);
    return hipGetLastError();
}

// The substeps of one time step: L launches of H_l <= kHMaxHalo substeps each
// (L = 2 for up to 2 kHMaxHalo substeps), through the scratch buffers 1 and 2,
// the last one writing buffer 0.  A single substep goes to buffer 1 and is
// copied back.
int heat_launches(int nsub) { return nsub <= 1 ? 1 : std::max(2, (nsub + kHMaxHalo - 1) / kHMaxHalo); }

hipError_t launch_heat_step(const DevState &s, const RunConst &rc, hipStream_t st) {
    if (rc.adi) return launch_adi_step(s, rc, st);
    const int L = heat_launches(s.nsub);
    int sub0 = 0, src = 0;
    for (int l = 0; l < L; ++l) {
        const int H = s.nsub / L + (l < s.nsub % L ? 1 : 0);
        const bool lastl = l == L - 1;
        const int dst = (lastl && s.nsub > 1) ? 0 : (src == 1 ? 2 : 1);
        const int Wd = kHT + 2 * H;
        const size_t lds = sizeof(double) * 4 * (size_t)Wd * Wd + sizeof(HeatRow) * (size_t)Wd;
        hipLaunchKernelGGL(k_heat_tile, dim3(s.nheat_blocks), dim3(256), lds, st, s, rc, src, dst, sub0, H,
                           lastl ? 1 : 0);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        sub0 += H;
        src = dst;
    }
    if (s.nsub == 1) {
        hipLaunchKernelGGL(k_copy2, dim3(blocks_for(s.N)), dim3(256), 0, st, s.u[1], s.T[1], s.u[0], s.T[0], s.N);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_finalize(const DevState &s, const RunConst &rc, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, st, s, rc);
    return hipGetLastError();
}

hipError_t launch_psi(const DevState &s, double *psi_out, hipStream_t st) {
    hipLaunchKernelGGL(k_psi, dim3(blocks_for(s.N)), dim3(256), 0, st, s, s.elem_coil, psi_out);
    return hipGetLastError();
}

hipError_t launch_gather(const double *src, const int *perm, int n, double *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n)), dim3(256), 0, st, src, perm, n, dst);
    return hipGetLastError();
}

hipError_t launch_scatter(const double *src, const int *perm, int n, double *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n)), dim3(256), 0, st, src, perm, n, dst);
    return hipGetLastError();
}

hipError_t launch_u_of_T(const DevState &s, const RunConst &rc, hipStream_t st) {
    hipLaunchKernelGGL(k_u_of_T, dim3(blocks_for(s.N)), dim3(256), 0, st, s, rc);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, double v, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_init_current(const DevState &s, hipStream_t st) {
    hipLaunchKernelGGL(k_init_current, dim3(blocks_for(s.N)), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_int, dim3(blocks_for(n)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_reset_scalars(Scalars *sc, double T_bath, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(64), 0, st, sc, T_bath);
    return hipGetLastError();
}

hipError_t launch_probe(const DevState &s, const double *zphys, int np, const double *pr, const double *pz,
                        double *br, double *bz, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe, dim3(blocks_for(np)), dim3(256), 0, st, s, zphys, np, pr, pz, br, bz);
    return hipGetLastError();
}

hipError_t launch_probe_chunked(const DevState &s, const double *zphys, int np, const double *pr, const double *pz,
                                double *br, double *bz, double2 *part, int nchunk, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    const int chunk = (s.N + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_probe_chunk, dim3(blocks_for(np), nchunk), dim3(256), 0, st, s, zphys, np, pr, pz, chunk,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_probe_sum, dim3(blocks_for(np)), dim3(256), 0, st, np, nchunk, pr, part, br, bz);
    return hipGetLastError();
}

hipError_t launch_stored(const DevState &s, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_stored, dim3(1), dim3(256), 0, st, s, out);
    return hipGetLastError();
}

// host copies of the elliptic approximations (test hook)
void host_ellip_f64(double m1, double *K, double *E) {
    const double L = -std::log(m1);
    *K = std::fma(ellipk64_Q(m1), L, ellipk64_P(m1));
    *E = std::fma(ellipe64_Q(m1), L, ellipe64_P(m1));
}
void host_ellip_f32(float m1, float *K, float *E) {
    const float L2 = -std::log2(m1);
    *K = std::fma(ellipk32_Q(m1), L2, ellipk32_P(m1));
    *E = std::fma(ellipe32_Q(m1), L2, ellipe32_P(m1));
}

}  // namespace coilq
