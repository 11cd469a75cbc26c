// coil_adjoint.hip -- kernels of the discrete adjoint of the coil time step.
//
// The objective is J = wQ Q + wT T_peak, Q the time-integrated Joule heat and
// T_peak the peak temperature over the run; parameters are the per-wire Jc
// multipliers c_w and the per-coil ramp rates.  Reverse of step k, given the
// adjoints (Ibar, ubar) of the state after the step:
//   1. ubar[e*] += wT / C(T_peak) when the peak was raised at step k+1;
//   2. qbar = wQ dt V, then each heat substep in reverse
//      (k_heat_adj: ubar <- ubar + T'(u) h_s [L(ubar/V) - G_b ubar/V],
//      qbar += h_s ubar);
//   3. k_wire_adj: the Joule source, the per-wire KKT system (same Cholesky
//      factor, transposed solve), the local law and Jc(B, T, c_w): produces
//      Ibar^k without the field term, the field weights Bbar, ubar += T'(u) Tbar,
//      and the c_w and transport-increment adjoints;
//   4. k_fieldT: Ibar^k += G^T Bbar, the transposed all-pairs field pass.
// Forward quantities of step k (I^k, B^k, dI, heat-substep temperatures) come
// from the recompute of the step's checkpoint segment.
#include <hip/hip_runtime.h>

#include "coil_adjoint.h"
#include "coil_device.h"

namespace coilq {

// ------------------------------------------------------------------ transposed field pass
// out_j = sum_e [ wr_e g_r(e, j) + wz_e g_z(e, j) ] over the elements e of
// j's coil; same work items, tiling and near/far split as the forward pass
// with the roles of targets and sources exchanged.
template <int MIXED>
__global__ __launch_bounds__(256) void k_fieldT(DevState s, RunConst rc, const double *wr,
                                                const double *wz, double *partT) {
    __shared__ float4 sp[kStage];   // (i_r, i_z, wr fp32, wz fp32)
    __shared__ double2 sw[kStage];  // (wr, wz) fp64
    const int tid = threadIdx.x;
    for (int it = blockIdx.x; it < s.nitems; it += gridDim.x) {
        const PairItem item = s.items[it];
        const CoilDev c = s.coils[item.coil];
        const int j = item.t0 + tid;
        const bool jact = tid < item.tn;
        const float2 jp = s.gpos[jact ? j : item.t0];
        const double jr = jp.x, jz = jp.y, c2j = c.c2d + jr;
        const float jr32 = jp.x, jz32 = jp.y, c2j32 = c.c2f + jp.x;
        const int wbase = item.t0 + (tid & ~63);
        const bool wact = wbase < item.t0 + item.tn;
        int4 jb = make_int4(0, 0, 0, 0);
        if (MIXED && wact) jb = s.bbox[c.group_off + (wbase - c.off) / kGroup];
        double nacc = 0.0;
        float fa = 0.f, ca = 0.f;
        const int send = item.s0 + item.sn;
        for (int s0 = item.s0; s0 < send; s0 += kStage) {
            const int cnt = min(kStage, send - s0);
            __syncthreads();
            for (int i = tid; i < cnt; i += blockDim.x) {
                const float2 p = s.gpos[s0 + i];
                const double a = wr[s0 + i], b = wz[s0 + i];
                sp[i] = make_float4(p.x, p.y, (float)a, (float)b);
                sw[i] = make_double2(a, b);
            }
            __syncthreads();
            if (!wact) continue;
            for (int g0 = 0; g0 < cnt; g0 += kGroup) {
                const int gn = min(kGroup, cnt - g0);
                bool near = true;
                if (MIXED) {
                    const int4 eb = s.bbox[c.group_off + (s0 + g0 - c.off) / kGroup];
                    near = groups_near(jb, eb, c.c2f, rc.m1_near);
                }
                if (near) {
#pragma unroll 4
                    for (int i = g0; i < g0 + gn; ++i) {
                        const float4 q = sp[i];
                        const double2 ww = sw[i];
                        pairT64((double)q.x - jr, (double)q.y - jz, c2j + (double)q.x, ww.x, ww.y, nacc);
                    }
                } else {
                    float pa = 0.f;
#pragma unroll 8
                    for (int i = g0; i < g0 + gn; ++i) {
                        const float4 q = sp[i];
                        pairT32(q.x - jr32, q.y - jz32, c2j32 + q.x, q.z, q.w, pa);
                    }
                    kahan_add(fa, ca, pa);
                }
            }
        }
        if (jact) partT[(size_t)item.chunk * s.N + j] = nacc + ((double)fa - (double)ca);
    }
}

// out[j] (+)= sum over the chunks of partT
__global__ void k_fieldT_sum(DevState s, const double *partT, double *out, int accumulate) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= s.N) return;
    const CoilDev c = s.coils[s.elem_coil[j]];
    const int nk = field_slots(s, c);
    double v = 0.0;
    int k = 0;
    for (; k + 16 <= nk; k += 16) {  // in order, 16 loads in flight
        double p[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) p[q] = partT[(size_t)(k + q) * s.N + j];
#pragma unroll
        for (int q = 0; q < 16; ++q) v += p[q];
    }
    for (; k < nk; ++k) v += partT[(size_t)k * s.N + j];
    out[j] = accumulate ? out[j] + v : v;
}

// field-transpose weights from a field adjoint: wr = Bbar_r kscale / rho, wz = Bbar_z kscale
__global__ void k_field_weights(DevState s, double *br, double *bz) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.N) return;
    const CoilDev c = s.coils[s.elem_coil[e]];
    br[e] = br[e] * c.kscale / s.rho[e];
    bz[e] = bz[e] * c.kscale;
}

// ------------------------------------------------------------------ wire + local law adjoint
__global__ __launch_bounds__(64) void k_wire_adj(DevState s, RunConst rc, AdjPtrs a) {
    extern __shared__ double sm[];
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const CoilDev c = s.coils[s.wire_coil[w]];
    const int lw = w - c.wire_off;
    const int layer = lw / c.turns;
    const int n = c.ne2;
    const bool act = lane < n;
    const int e = c.off + lw * n + (act ? lane : 0);
    const double dt = rc.dt;
    const double d2 = c.d * c.d;
    const double I0 = a.I[e], T = a.T[e], br = a.Br[e], bz = a.Bz[e];
    const double dI = act ? a.dI[e] : 0.0;
    const double cw = s.cw[w];
    Local lo;
    if (act) {
        local_law(rc, cw, s.jcs[e], I0 / d2, T, br, bz, lo);
    } else {
        lo.Jc = lo.x = lo.E = lo.Ep = lo.fT = lo.fB = lo.Bm = lo.p = 0.0;
    }
    const double re = s.r[e];
    const double kap = 2.0 * kPi * re / d2;
    const size_t lay = (size_t)(c.layer_off + layer);
    const double *M = s.Mlay + lay * n * n;
    const double diag_add = dt * kap * lo.Ep;
    const double I1 = I0 + dI;
    const double Elin = lo.E + lo.Ep * dI / d2;
    const double qb = act ? a.qbar[e] : 0.0;
    const double Ib1 = act ? a.Ibar[e] : 0.0;
    // adjoint of dI: through I^{k+1} = I^k + dI and through q
    double xv = act ? Ib1 + qb * (lo.Ep * I1 / (d2 * d2) + Elin / d2) : 0.0;
    double yv, sy;
    // A = M + dt diag(kap E') is symmetric: the same solves as the forward step,
    // with the layer's inverse when the diagonal addition vanishes in FP64
    const double mee = act ? M[(size_t)lane * n + lane] : 1.0;
    if (__all(act ? (mee + diag_add == mee) : 1)) {
        xv = matvec_cols(s.Minv + lay * n * n, n, lane, act, xv);
        yv = act ? s.yl[lay * n + lane] : 0.0;
        sy = s.syl[lay];
    } else {
        load_wire_matrix(sm, M, n, lane, act, diag_add);
        chol_lds(sm, n, lane, act, sm + packed_size(n));
        yv = act ? 1.0 : 0.0;
        solve2_lds(sm, n, lane, act, xv, yv);
        sy = wave_sum(act ? yv : 0.0);
    }
    const double sx = wave_sum(act ? xv : 0.0);
    const double numu = sx / sy;  // adjoint of the net-current constraint
    const double nu = act ? xv - numu * yv : 0.0;
    // adjoints of E and E' (through b, the matrix diagonal and q)
    const double Eb = act ? qb * I1 / d2 - dt * 2.0 * kPi * re * nu : 0.0;
    const double Epb = act ? qb * (dI / d2) * (I1 / d2) - nu * dI * dt * kap : 0.0;
    const double dItb = wave_sum(act ? -s.psi[e] * nu : 0.0) + numu;
    // local law (E, E' as functions of J and Jc)
    double Jb = 0.0, Jcb = 0.0;
    if (act) local_law_adj(rc, lo, I0 / d2, Eb, Epb, Jb, Jcb);
    if (act) a.Ibar[e] = Ib1 + qb * Elin / d2 + Jb / d2;
    // Jc = c_w jcs fT fB
    const double cwb = wave_sum(act ? Jcb * s.jcs[e] * lo.fT * lo.fB : 0.0);
    const double Tb = (act && T < rc.Tc) ? Jcb * cw * s.jcs[e] * lo.fB * (-1.0 / rc.Tc) : 0.0;
    const double Bmb = act ? Jcb * (-lo.Jc / (rc.B0 + lo.Bm)) : 0.0;
    double Brb = 0.0, Bzb = 0.0;
    if (lo.Bm > 0.0) {
        Brb = Bmb * br / lo.Bm;
        Bzb = Bmb * bz / lo.Bm;
    }
    if (act) {
        a.wr[e] = Brb * c.kscale / s.rho[e];
        a.wz[e] = Bzb * c.kscale;
        if (Tb != 0.0) a.ubar[e] += Tb / (rc.C0 * pow(T / rc.T_ref, rc.cp_exp));
    }
    if (lane == 0) {
        a.cbar[w] += cwb;
        a.dItbar[w] += dItb;
    }
}

// ------------------------------------------------------------------ heat adjoint (one substep)
__global__ __launch_bounds__(256) void k_heat_adj(DevState s, RunConst rc, const double *ub_in,
                                                  double *ub_out, const double *Tsub, double *qbar,
                                                  double hs) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.N) return;
    const double ue = ub_in[e];
    const double we = ue * s.invV[e];
    double tb = -s.Gb[e] * we;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int nbr = s.nb[4 * e + f];
        if (nbr >= 0) tb += s.G[4 * e + f] * (ub_in[nbr] * s.invV[nbr] - we);
    }
    tb *= hs;
    const double Ts = Tsub[e];
    ub_out[e] = ue + tb / (rc.C0 * pow(Ts / rc.T_ref, rc.cp_exp));
    qbar[e] += hs * ue;
}

__global__ void k_qbar_init(DevState s, double *qbar, double wQdt) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < s.N) qbar[e] = wQdt * s.V[e];
}

__global__ void k_add_at(double *p, int i, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[i] += v;
}

__global__ void k_set_step(Scalars *sc, long long step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->step = step;
}

__global__ void k_copy(const double *src, double *dst, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------ launchers
static inline int nblk(int n) { return (n + 255) / 256; }

hipError_t launch_fieldT(const DevState &s, const RunConst &rc, int grid_limit, const double *wr,
                         const double *wz, double *partT, hipStream_t st) {
    if (s.nitems == 0) return hipSuccess;
    const int grid = grid_limit > 0 ? min(grid_limit, s.nitems) : s.nitems;
    if (rc.prec == COIL_MIXED)
        hipLaunchKernelGGL(k_fieldT<1>, dim3(grid), dim3(s.tile_targets), 0, st, s, rc, wr, wz, partT);
    else
        hipLaunchKernelGGL(k_fieldT<0>, dim3(grid), dim3(s.tile_targets), 0, st, s, rc, wr, wz, partT);
    return hipGetLastError();
}

hipError_t launch_fieldT_sum(const DevState &s, const double *partT, double *out, int accumulate,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_fieldT_sum, dim3(nblk(s.N)), dim3(256), 0, st, s, partT, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_field_weights(const DevState &s, double *br, double *bz, hipStream_t st) {
    hipLaunchKernelGGL(k_field_weights, dim3(nblk(s.N)), dim3(256), 0, st, s, br, bz);
    return hipGetLastError();
}

hipError_t launch_wire_adj(const DevState &s, const RunConst &rc, const AdjPtrs &a, hipStream_t st) {
    const size_t lds = sizeof(double) * ((size_t)packed_size(s.max_ne2) + kCholPad);
    hipLaunchKernelGGL(k_wire_adj, dim3(s.Nw), dim3(64), lds, st, s, rc, a);
    return hipGetLastError();
}

hipError_t launch_heat_adj(const DevState &s, const RunConst &rc, const double *ub_in, double *ub_out,
                           const double *Tsub, double *qbar, hipStream_t st) {
    const double hs = rc.dt / (double)s.nsub;
    hipLaunchKernelGGL(k_heat_adj, dim3(nblk(s.N)), dim3(256), 0, st, s, rc, ub_in, ub_out, Tsub, qbar, hs);
    return hipGetLastError();
}

hipError_t launch_qbar_init(const DevState &s, double *qbar, double wQdt, hipStream_t st) {
    hipLaunchKernelGGL(k_qbar_init, dim3(nblk(s.N)), dim3(256), 0, st, s, qbar, wQdt);
    return hipGetLastError();
}

hipError_t launch_add_at(double *p, int i, double v, hipStream_t st) {
    hipLaunchKernelGGL(k_add_at, dim3(1), dim3(64), 0, st, p, i, v);
    return hipGetLastError();
}

hipError_t launch_set_step(Scalars *sc, long long step, hipStream_t st) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, st, sc, step);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace coilq
