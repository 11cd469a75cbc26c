// coil_coupled.hip -- fully coupled A-V solve of one time step
// (COIL_COUPLE_FULL).
//
// Every ring e of a coil obeys 2 pi r_e E_e + U_w(e) = -dPhi_e/dt with the
// flux of ALL element currents of the coil (paper, Methods, "Numerical
// Algorithm": the field of every subelement is updated from the net currents
// of all subelements until the iteration has converged).  Linearised backward
// Euler:
//   A dI + dt P U = b,  P^T dI = dI_t 1,
//   A = M + dt diag(2 pi r E'/d^2),  b = -pi r^2 dB_a - dt 2 pi r E,
// M the coil's inductance matrix, P the element-to-wire incidence.
// The step first solves each wire with the other wires' transport current
// only (the per-wire kernels, which also store each factorised wire block);
// that dI_0 meets the constraints.  The correction x (zero net current per
// wire) minimises the energy of A on that subspace: conjugate gradients with
// the per-wire constrained inverse
//   S_w r = A_ww^-1 r - A_ww^-1 1 (1^T A_ww^-1 r) / (1^T A_ww^-1 1)
// as preconditioner (it maps onto the subspace and removes the range of P),
// and the translation-reuse flux pass for the off-diagonal part of A.  The
// residual r = b - A dI keeps a per-wire constant part (dt U_w at
// convergence) that S annihilates only by cancellation; it is moved out of r
// into a per-wire sum c_w after every update, which leaves the iteration
// unchanged in exact arithmetic and keeps S r accurate.  The iteration stops
// when r^T S r <= cg_tol^2 r_0^T S r_0.  Then dI = dI_0 + x,
// U_w = (c_w + 1^T A_ww^-1 r / 1^T A_ww^-1 1) / dt, and the flux update
// M dI + pi r^2 dB_a = -dt 2 pi r E_lin - (r + c_w) (from A dI = b - r).
#include <hip/hip_runtime.h>

#include <climits>

#include "coil_coupled.h"
#include "coil_device.h"
#include "coil_field_tz.h"

namespace coilq {

// v (internal order) -> vpub (public order), clearing the flux pass's ticket.
// mode 1: first p = z + beta p (the next search direction).  Skipped once the
// iteration has converged.
__global__ void k_cg_prep(DevState s, const double *v_in, double *vpub, int *ticket, int mode) {
    if (s.cg->done) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < s.N) {
        double v;
        if (mode == 1) {
            v = s.cg_z[i] + s.cg->beta * s.cg_p[i];
            s.cg_p[i] = v;
        } else {
            v = v_in[i];
        }
        vpub[s.perm[i]] = v;
    }
    if (ticket && i == 0) *ticket = 0;
}

// A v = (off-diagonal flux from the partial sums) + (L_self + dt D) v.
// mode 0: r = b - A dI_0; mode 1: q = A p and per-block sums of p.q.
__global__ __launch_bounds__(256) void k_cg_av(DevState s, RunConst rc, int mode) {
    __shared__ double red[256];
    if (s.cg->done) return;
    const int tid = threadIdx.x;
    const int e = blockIdx.x * 256 + tid;
    double pq = 0.0;
    if (e < s.N) {
        const CoilDev c = s.coils[s.elem_coil[e]];
        const int nk = s.flux_fft ? 1 : c.nslot_tz;
        double off = 0.0;
        for (int k = 0; k < nk; ++k) off += s.part[(size_t)k * s.N + e].y;
        const double re = s.r[e];
        const double diag = s.Lself[e] + rc.dt * 2.0 * kPi * re * s.Ep[e] / (c.d * c.d);
        if (mode == 0) {
            const double v = s.dI[e];
            const double b = -kPi * re * re * (rc.dBa_dt * rc.dt) - rc.dt * 2.0 * kPi * re * s.E[e];
            s.cg_r[e] = b - (off + diag * v);
        } else {
            const double p = s.cg_p[e];
            const double q = off + diag * p;
            s.cg_q[e] = q;
            pq = p * q;
        }
    }
    if (mode == 0) return;
    red[tid] = pq;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) s.cg_red[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_cg_alpha(DevState s, int nblocks) {
    __shared__ double red[256];
    if (s.cg->done) return;
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int b = tid; b < nblocks; b += 256) v += s.cg_red[b];
    red[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) s.cg->alpha = red[0] > 0.0 ? s.cg->rho / red[0] : 0.0;
}

// A_ww^-1 v and A_ww^-1 1 of wire w (lane i holds element i), with the
// layer's inverse when the resistive diagonal vanishes in FP64 (as in the
// per-wire kernels), else with the wire's Cholesky factor stored this step.
__device__ __forceinline__ void wire_inverse(const DevState &s, const RunConst &rc, const CoilDev &c, int w,
                                             int lane, bool act, int e, double v, double *sm, double &xv,
                                             double &yv, double &sy) {
    const int n = c.ne2;
    const int lw = w - c.wire_off;
    const size_t lay = (size_t)(c.layer_off + lw / c.turns);
    const double *M = s.Mlay + lay * n * n;
    const double diag_add = act ? rc.dt * 2.0 * kPi * s.r[e] * s.Ep[e] / (c.d * c.d) : 0.0;
    const double mee = act ? M[(size_t)lane * n + lane] : 1.0;
    if (__all(act ? (mee + diag_add == mee) : 1)) {
        xv = matvec_cols(s.Minv + lay * n * n, n, lane, act, v);
        yv = act ? s.yl[lay * n + lane] : 0.0;
        sy = s.syl[lay];
    } else {
        // the factor into LDS eight values per lane at a time, their loads
        // issued together (a loop that stores each value as it arrives pays
        // the memory latency once per value: 33 times at n_e = 64); loads
        // past the end re-read the last
        const double *L = s.cg_L + (size_t)w * packed_size(s.max_ne2);
        const int np = packed_size(n);
        for (int b = 0; b < np; b += 8 * 64) {
            double f[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) f[k] = L[min(b + lane + 64 * k, np - 1)];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (b + lane + 64 * k < np) sm[b + lane + 64 * k] = f[k];
        }
        __syncthreads();
        xv = v;
        yv = act ? 1.0 : 0.0;
        solve2_lds(sm, n, lane, act, xv, yv);
        sy = wave_sum(act ? yv : 0.0);
    }
}

// One wave per wire.  mode 0: x = 0, z = S r, p = z; mode 1: x += alpha p,
// r -= alpha q, z = S r; in both the wire's mean of r moves to c_w first.
// Per-wire sums of r.z.
__global__ __launch_bounds__(64) void k_cg_wire(DevState s, RunConst rc, int mode) {
    extern __shared__ double sm[];
    if (s.cg->done) return;
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const CoilDev c = s.coils[s.wire_coil[w]];
    const int n = c.ne2;
    const bool act = lane < n;
    const int e = c.off + (w - c.wire_off) * n + (act ? lane : 0);
    double r = 0.0;
    if (act) {
        if (mode == 0) {
            s.cg_x[e] = 0.0;
            r = s.cg_r[e];
        } else {
            const double a = s.cg->alpha;
            s.cg_x[e] += a * s.cg_p[e];
            r = s.cg_r[e] - a * s.cg_q[e];
        }
    }
    const double mean = wave_sum(r) / (double)n;
    r = act ? r - mean : 0.0;
    if (act) s.cg_r[e] = r;
    if (lane == 0) s.cg_cw[w] = (mode == 0 ? 0.0 : s.cg_cw[w]) + mean;
    double xv, yv, sy;
    wire_inverse(s, rc, c, w, lane, act, e, r, sm, xv, yv, sy);
    const double sx = wave_sum(act ? xv : 0.0);
    const double z = act ? xv - (sx / sy) * yv : 0.0;
    if (act) {
        s.cg_z[e] = z;
        if (mode == 0) s.cg_p[e] = z;
    }
    const double rz = wave_sum(act ? r * z : 0.0);
    if (lane == 0) s.cg_rw[w] = rz;
}

__global__ __launch_bounds__(256) void k_cg_beta(DevState s, int mode) {
    __shared__ double red[256];
    if (s.cg->done) return;
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int w = tid; w < s.Nw; w += 256) v += s.cg_rw[w];
    red[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        CgScalars *g = s.cg;
        const double rho = red[0];
        if (mode == 0) {
            g->rho0 = rho;
            g->beta = 0.0;
            g->iters = 0;
        } else {
            g->beta = g->rho > 0.0 ? rho / g->rho : 0.0;
            g->iters += 1;
        }
        g->rho = rho;
        if (!(rho > g->tol2 * g->rho0) || g->iters >= g->maxit) g->done = 1;
    }
}

// dI = dI_0 + x and the step's updates (as the per-wire kernel makes them
// for the transport-only drive): I, the Joule source, the flux, U_w, Q_w.
__global__ __launch_bounds__(64) void k_cg_finish(DevState s, RunConst rc) {
    extern __shared__ double sm[];
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const CoilDev c = s.coils[s.wire_coil[w]];
    const int n = c.ne2;
    const bool act = lane < n;
    const int e = c.off + (w - c.wire_off) * n + (act ? lane : 0);
    const double dt = rc.dt;
    const double d2 = c.d * c.d;
    const double r = act ? s.cg_r[e] : 0.0;
    double xv, yv, sy;
    wire_inverse(s, rc, c, w, lane, act, e, r, sm, xv, yv, sy);
    const double sx = wave_sum(act ? xv : 0.0);
    const double cw = s.cg_cw[w];
    const double U = (cw + sx / sy) / dt;
    double qv = 0.0;
    unsigned bad = 0u;
    if (act) {
        const double dI = s.dI[e] + s.cg_x[e];
        const double I1 = s.I[e] + dI;
        const double E = s.E[e], Ep = s.Ep[e], re = s.r[e];
        const double Elin = E + Ep * dI / d2;
        qv = Elin * (I1 / d2);
        s.Phi[e] += -dt * 2.0 * kPi * re * Elin - (r + cw);
        s.I[e] = I1;
        s.dI[e] = dI;
        s.q[e] = qv;
        if (s.rec_dI) s.rec_dI[e] = dI;
        if (!isfinite(I1) || !isfinite(qv)) bad = ST_NONFINITE;
    }
    const double qw = wave_sum(act ? dt * s.V[e] * qv : 0.0);
    bad = wave_or(bad);
    if (lane == 0) {
        s.Uw[w] = U;
        s.wq[w] = qw;
        s.Qw[w] += qw;
        if (bad) atomicOr(&s.sc->status, bad);
    }
}

__global__ void k_cg_reset(CgScalars *g, double tol2, int maxit) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        g->rho = g->rho0 = g->alpha = g->beta = 0.0;
        g->tol2 = tol2;
        g->iters = 0;
        g->maxit = maxit;
        g->done = 0;
    }
}

static inline int blocks256(int n) { return (n + 255) / 256; }

hipError_t launch_cg_begin(const DevState &s, const RunConst &rc, const TzPlan &tp, const FftPlan &fp, double *vpub,
                           const int *pub2int, double tol, int maxit, hipStream_t st) {
    const size_t lds = sizeof(double) * (size_t)packed_size(s.max_ne2);
    hipLaunchKernelGGL(k_cg_reset, dim3(1), dim3(64), 0, st, s.cg, tol * tol, maxit);
    hipLaunchKernelGGL(k_cg_prep, dim3(blocks256(s.N)), dim3(256), 0, st, s, (const double *)s.dI, vpub, tp.ticket, 0);
    hipError_t e = s.flux_fft ? launch_flux_fft(s, fp, s.dI, pub2int, &s.cg->done, st)
                              : launch_flux_tz(s, rc, tp, vpub, pub2int, &s.cg->done, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cg_av, dim3(blocks256(s.N)), dim3(256), 0, st, s, rc, 0);
    hipLaunchKernelGGL(k_cg_wire, dim3(s.Nw), dim3(64), lds, st, s, rc, 0);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, s, 0);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const DevState &s, const RunConst &rc, const TzPlan &tp, const FftPlan &fp,
                               double *vpub, const int *pub2int, hipStream_t st) {
    const size_t lds = sizeof(double) * (size_t)packed_size(s.max_ne2);
    hipLaunchKernelGGL(k_cg_prep, dim3(blocks256(s.N)), dim3(256), 0, st, s, (const double *)nullptr, vpub, tp.ticket,
                       1);
    // the new direction p (k_cg_prep) in internal order for the fast convolution
    hipError_t e = s.flux_fft ? launch_flux_fft(s, fp, s.cg_p, pub2int, &s.cg->done, st)
                              : launch_flux_tz(s, rc, tp, vpub, pub2int, &s.cg->done, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cg_av, dim3(blocks256(s.N)), dim3(256), 0, st, s, rc, 1);
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, st, s, blocks256(s.N));
    hipLaunchKernelGGL(k_cg_wire, dim3(s.Nw), dim3(64), lds, st, s, rc, 1);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, s, 1);
    return hipGetLastError();
}

hipError_t launch_cg_finish(const DevState &s, const RunConst &rc, hipStream_t st) {
    const size_t lds = sizeof(double) * (size_t)packed_size(s.max_ne2);
    hipLaunchKernelGGL(k_cg_finish, dim3(s.Nw), dim3(64), lds, st, s, rc);
    return hipGetLastError();
}

}  // namespace coilq
