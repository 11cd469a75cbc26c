// coil_adi.hip -- alternating-direction implicit heat step (COIL_HEAT_ADI).
//
// Peaceman-Rachford on the finite volumes of each coil's (r, z) grid (paper,
// Methods, heat paragraph: ADI on the composite coil, c, kappa and h
// proportional to T^3).  With the coefficients at T^n and the Joule source q
// held, L_r and L_z the radial and axial parts of the net inflow (borders
// included):
//   V C (T* - T^n) / (dt/2) = L_r(T*) + L_z(T^n) + V q     (one system per column)
//   V C (T** - T*) / (dt/2) = L_r(T*) + L_z(T**) + V q     (one system per row)
//   u^{n+1} = u^n + (dt/V) [L_r(T*) + (L_z(T^n) + L_z(T**))/2] + dt q,
//   T^{n+1} = T(u^{n+1}).
// Face conductances G = A / (d/(2 k_e) + d/(2 k_f) + R_ins) with
// k = k0 (T/T_ref)^k_exp k_mult and R_ins = ins_R0 (T_ref/T_face)^k_exp on
// faces between wires; border G^b = A / (1/h + d/(2 k_e)), h = h0 (T/T_ref)^h_exp.
// Both sides of a face evaluate the same symmetric expression, so the
// interior fluxes cancel bitwise and the energy balance is exact.
// Three kernels: the coefficients (per element), the radial sweep (one
// workgroup per grid column) and the axial sweep with the enthalpy update
// (one workgroup per grid row); each sweep solves its tridiagonal system by
// parallel cyclic reduction in LDS.
#include <hip/hip_runtime.h>

#include <climits>

#include "coil_device.h"

namespace coilq {

constexpr int kAdiThreads = 256;
constexpr int kAdiPerThread = 6;  // lines of at most kAdiThreads * kAdiPerThread = 1536 cells

__device__ __forceinline__ int elem_at(const CoilDev &c, int ir, int iz) {
    return c.off + ((ir / c.ne) * c.turns + iz / c.ne) * c.ne2 + (ir % c.ne) * c.ne + iz % c.ne;
}

__device__ __forceinline__ double k_of(const RunConst &rc, double T, double km) {
    return rc.k0 * (rc.k_exp == 0.0 ? 1.0 : pow(T / rc.T_ref, rc.k_exp)) * km;
}

// the coil of line (column or row) b: the last coil whose first line is <= b
__device__ __forceinline__ int coil_of_line(const DevState &s, int b, bool rows) {
    int lo = 0, hi = s.ncoils - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        const int first = rows ? s.coils[mid].row_off : s.coils[mid].col_off;
        if (first <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Coefficients at T^n: C V, the four face conductances (inner, outer, lower,
// upper; 0 on borders), the radial and axial border conductances, L_z(T^n).
__global__ __launch_bounds__(256) void k_adi_coef(DevState s, RunConst rc) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.N) return;
    const CoilDev c = s.coils[s.elem_coil[e]];
    const float2 gp = s.gpos[e];
    const int ir = (int)gp.x;
    const HeatRow R = s.hrow[c.row_off + ir];
    const double *T = s.T[0];
    const double Te = T[e];
    const double ke = k_of(rc, Te, s.kmult[e]);
    const double he = c.d / (2.0 * ke);
    const int we = (e - c.off) / c.ne2;
    s.adi_Cv[e] = s.V[e] * rc.C0 * pow(Te / rc.T_ref, rc.cp_exp);
    const double area[4] = {R.ain, R.aout, R.aax, R.aax};
    double gbr = 0.0, gbz = 0.0, lz = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int n = s.nb[4 * e + f];
        double G = 0.0;
        if (n >= 0) {
            const double Tn = T[n];
            const double hn = c.d / (2.0 * k_of(rc, Tn, s.kmult[n]));
            double Rf = he + hn;
            if (rc.ins_R0 > 0.0 && (n - c.off) / c.ne2 != we)
                Rf += rc.ins_R0 * (rc.k_exp == 0.0 ? 1.0 : pow(rc.T_ref / (0.5 * (Te + Tn)), rc.k_exp));
            G = area[f] / Rf;
            if (f >= 2) lz += G * (Tn - Te);
        } else if (rc.h0 > 0.0) {
            const double h = rc.h0 * (rc.h_exp == 0.0 ? 1.0 : pow(Te / rc.T_ref, rc.h_exp));
            const double gb = area[f] / (1.0 / h + he);
            if (f < 2) gbr += gb;
            else gbz += gb;
        }
        s.adi_G[4 * (size_t)e + f] = G;
    }
    s.adi_Gbr[e] = gbr;
    s.adi_Gbz[e] = gbz;
    s.adi_Lz0[e] = gbz * (rc.T_bath - Te) + lz;
}

// Parallel cyclic reduction of a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i
// (i < n <= 1536, diagonally dominant) held in LDS; x_i returned in d.
__device__ void pcr_solve(double *a, double *b, double *c, double *d, int n) {
    const int tid = threadIdx.x;
    for (int sft = 1; sft < n; sft <<= 1) {
        double na[kAdiPerThread], nb[kAdiPerThread], nc[kAdiPerThread], nd[kAdiPerThread];
#pragma unroll
        for (int k = 0; k < kAdiPerThread; ++k) {
            const int i = tid + k * kAdiThreads;
            if (i < n) {
                const int lo = i - sft, hi = i + sft;
                double k1 = 0.0, k2 = 0.0, al = 0.0, cl = 0.0, dl = 0.0, ah = 0.0, ch = 0.0, dh = 0.0;
                if (lo >= 0) {
                    k1 = a[i] / b[lo];
                    al = a[lo];
                    cl = c[lo];
                    dl = d[lo];
                }
                if (hi < n) {
                    k2 = c[i] / b[hi];
                    ah = a[hi];
                    ch = c[hi];
                    dh = d[hi];
                }
                na[k] = -al * k1;
                nc[k] = -ch * k2;
                nb[k] = b[i] - cl * k1 - ah * k2;
                nd[k] = d[i] - dl * k1 - dh * k2;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kAdiPerThread; ++k) {
            const int i = tid + k * kAdiThreads;
            if (i < n) {
                a[i] = na[k];
                b[i] = nb[k];
                c[i] = nc[k];
                d[i] = nd[k];
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += kAdiThreads) d[i] = d[i] / b[i];
    __syncthreads();
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int o = kAdiThreads / 2; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// radial half step: workgroup b solves grid column b (coil, i_z) for T*, then
// L_r(T*) and the column's radial border outflow
__global__ __launch_bounds__(kAdiThreads) void k_adi_r(DevState s, RunConst rc) {
    extern __shared__ double sh[];
    __shared__ double red[kAdiThreads];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    if (b >= s.adi_ncols) {
        if (tid == 0) s.hb_out[b] = 0.0;
        return;
    }
    const CoilDev c = s.coils[coil_of_line(s, b, false)];
    const int iz = b - c.col_off;
    const int n = c.layers * c.ne;
    double *A = sh, *B = sh + n, *Cc = sh + 2 * n, *D = sh + 3 * n;
    const double dt = rc.dt;
    for (int i = tid; i < n; i += kAdiThreads) {
        const int e = elem_at(c, i, iz);
        const double m = 2.0 * s.adi_Cv[e] / dt;
        const double g0 = s.adi_G[4 * (size_t)e], g1 = s.adi_G[4 * (size_t)e + 1], gb = s.adi_Gbr[e];
        A[i] = -g0;
        Cc[i] = -g1;
        B[i] = m + g0 + g1 + gb;
        D[i] = m * s.T[0][e] + s.adi_Lz0[e] + s.V[e] * s.q[e] + gb * rc.T_bath;
    }
    __syncthreads();
    pcr_solve(A, B, Cc, D, n);
    double out = 0.0;
    for (int i = tid; i < n; i += kAdiThreads) {
        const int e = elem_at(c, i, iz);
        const double x = D[i], gb = s.adi_Gbr[e];
        double lr = gb * (rc.T_bath - x);
        if (i > 0) lr += s.adi_G[4 * (size_t)e] * (D[i - 1] - x);
        if (i < n - 1) lr += s.adi_G[4 * (size_t)e + 1] * (D[i + 1] - x);
        s.adi_Ts[e] = x;
        s.adi_Lr1[e] = lr;
        out += dt * gb * (x - rc.T_bath);
    }
    const double o = block_sum(out, red);
    if (tid == 0) s.hb_out[b] = o;
}

// axial half step: workgroup b solves grid row b (coil, i_r) for T**, then the
// enthalpy and temperature of the step, the row's axial border outflow and its
// largest T (lowest public index on ties)
__global__ __launch_bounds__(kAdiThreads) void k_adi_z(DevState s, RunConst rc) {
    extern __shared__ double sh[];
    __shared__ double red[kAdiThreads];
    __shared__ double red_t[kAdiThreads];
    __shared__ long long red_i[kAdiThreads];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    double *hb2 = s.hb_out + s.nheat_blocks;
    if (b >= s.adi_nrows) {
        if (tid == 0) {
            hb2[b] = 0.0;
            s.hb_max[b] = -INFINITY;
            s.hb_arg[b] = LLONG_MAX;
        }
        return;
    }
    const CoilDev c = s.coils[coil_of_line(s, b, true)];
    const int ir = b - c.row_off;
    const int n = c.turns * c.ne;
    const int nz = n;
    double *A = sh, *B = sh + n, *Cc = sh + 2 * n, *D = sh + 3 * n;
    const double dt = rc.dt;
    for (int j = tid; j < n; j += kAdiThreads) {
        const int e = elem_at(c, ir, j);
        const double m = 2.0 * s.adi_Cv[e] / dt;
        const double g2 = s.adi_G[4 * (size_t)e + 2], g3 = s.adi_G[4 * (size_t)e + 3], gb = s.adi_Gbz[e];
        A[j] = -g2;
        Cc[j] = -g3;
        B[j] = m + g2 + g3 + gb;
        D[j] = m * s.adi_Ts[e] + s.adi_Lr1[e] + s.V[e] * s.q[e] + gb * rc.T_bath;
    }
    __syncthreads();
    pcr_solve(A, B, Cc, D, n);
    double out = 0.0, tm = -INFINITY;
    long long ti = LLONG_MAX;
    unsigned bad = 0u;
    for (int j = tid; j < n; j += kAdiThreads) {
        const int e = elem_at(c, ir, j);
        const double y = D[j], gb = s.adi_Gbz[e];
        double lz = gb * (rc.T_bath - y);
        if (j > 0) lz += s.adi_G[4 * (size_t)e + 2] * (D[j - 1] - y);
        if (j < n - 1) lz += s.adi_G[4 * (size_t)e + 3] * (D[j + 1] - y);
        const double Tn = s.T[0][e];
        const double un = s.u[0][e] + dt * s.invV[e] * (s.adi_Lr1[e] + 0.5 * (s.adi_Lz0[e] + lz)) + dt * s.q[e];
        const double Tv = T_of_u(rc, un);
        s.u[0][e] = un;
        s.T[0][e] = Tv;
        out += dt * 0.5 * gb * ((Tn - rc.T_bath) + (y - rc.T_bath));
        if (!isfinite(Tv)) bad = ST_NONFINITE;
        const long long pub = (long long)c.off + (long long)ir * nz + j;
        if (Tv > tm || (Tv == tm && pub < ti)) {
            tm = Tv;
            ti = pub;
        }
    }
    if (bad) atomicOr(&s.sc->status, bad);
    const double o = block_sum(out, red);
    red_t[tid] = tm;
    red_i[tid] = ti;
    __syncthreads();
    for (int k = kAdiThreads / 2; k > 0; k >>= 1) {
        if (tid < k) {
            const double x = red_t[tid], y2 = red_t[tid + k];
            if (y2 > x || (y2 == x && red_i[tid + k] < red_i[tid])) {
                red_t[tid] = y2;
                red_i[tid] = red_i[tid + k];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        hb2[b] = o;
        s.hb_max[b] = red_t[0];
        s.hb_arg[b] = red_i[0];
    }
}

hipError_t launch_adi_step(const DevState &s, const RunConst &rc, hipStream_t st) {
    hipLaunchKernelGGL(k_adi_coef, dim3((s.N + 255) / 256), dim3(256), 0, st, s, rc);
    const size_t lds = 4 * sizeof(double) * (size_t)s.adi_maxline;
    hipLaunchKernelGGL(k_adi_r, dim3(s.nheat_blocks), dim3(kAdiThreads), lds, st, s, rc);
    hipLaunchKernelGGL(k_adi_z, dim3(s.nheat_blocks), dim3(kAdiThreads), lds, st, s, rc);
    return hipGetLastError();
}

}  // namespace coilq
