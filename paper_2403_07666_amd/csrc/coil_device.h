// coil_device.h -- device functions shared by the forward and adjoint
// kernels: the ring-field pair (FP64 and FP32 forms, forward and transposed),
// the local power law, the wire matrix factorisation and solves in LDS.
// Forward and adjoint call the same functions, so a recomputed forward
// quantity is bitwise the one the forward pass produced.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "coil_internal.h"
#include "ellip_coeffs.h"

namespace coilq {

// ------------------------------------------------------------------ helpers
// Wavefront reductions (every lane of the wave active), the result in every
// lane.  DPP moves in registers: pairs and quads by quad permutations, 8 and
// 16 lanes by the half-row and row mirrors, then rows 1 and 3 take row 0 and
// 2 (broadcast of lane 15) and rows 2 and 3 take rows 0-1 (broadcast of lane
// 31); lane 63 then holds the result, read back as a scalar.  A butterfly of
// lane shuffles instead goes through the LDS crossbar at each of its six
// steps.  A 64-bit value moves as two 32-bit halves; lanes a row mask leaves
// out receive `old` (the operation's identity).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_mov64(double x, double old) {
    const long long b = __double_as_longlong(x), o = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffLL), (int)(b & 0xffffffffLL), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane63(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov64<0xb1, 0xf>(v, 0.0);   // quad_perm [1, 0, 3, 2]
    v += dpp_mov64<0x4e, 0xf>(v, 0.0);   // quad_perm [2, 3, 0, 1]
    v += dpp_mov64<0x141, 0xf>(v, 0.0);  // row_half_mirror
    v += dpp_mov64<0x140, 0xf>(v, 0.0);  // row_mirror
    v += dpp_mov64<0x142, 0xa>(v, 0.0);  // row_bcast:15 into rows 1, 3
    v += dpp_mov64<0x143, 0xc>(v, 0.0);  // row_bcast:31 into rows 2, 3
    return lane63(v);
}
__device__ __forceinline__ double wave_max(double v) {
    const double lo = -INFINITY;
    v = fmax(v, dpp_mov64<0xb1, 0xf>(v, lo));
    v = fmax(v, dpp_mov64<0x4e, 0xf>(v, lo));
    v = fmax(v, dpp_mov64<0x141, 0xf>(v, lo));
    v = fmax(v, dpp_mov64<0x140, 0xf>(v, lo));
    v = fmax(v, dpp_mov64<0x142, 0xa>(v, lo));
    v = fmax(v, dpp_mov64<0x143, 0xc>(v, lo));
    return lane63(v);
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// FP64 pair: adds the (B_r * rho_t, B_z) contribution of a source of strength
// sv (= mu0 I / (2 pi d)) at grid offsets (dr, dz), sr = rho_t + rho_s.
__device__ __forceinline__ void pair64(double dr, double dz, double sr, double sv, double &ar,
                                       double &az) {
    const double dz2 = dz * dz;
    const double al2 = fma(dr, dr, dz2);
    const double be2 = fma(sr, sr, dz2);
    const double rb = rsqrt(be2);
    const double m1 = al2 * (rb * rb);
    const double L = -log(m1);
    const double K = fma(ellipk64_Q(m1), L, ellipk64_P(m1));
    const double E = fma(ellipe64_Q(m1), L, ellipe64_P(m1));
    const double f = sv * rb / al2;
    const double alK = al2 * K;
    const double gz = fma(fma(-dr, sr, -dz2), E, alK);
    const double gr = dz * fma(0.5 * (al2 + be2), E, -alK);
    const bool ok = al2 > 0.0;  // the element's own ring is excluded
    az = ok ? fma(f, gz, az) : az;
    ar = ok ? fma(f, gr, ar) : ar;
}

// FP32 pair (far field): same formula; -log2(m1), rsqrt, rcp in hardware.
__device__ __forceinline__ void pair32(float dr, float dz, float sr, float sv, float &ar,
                                       float &az) {
    const float dz2 = dz * dz;
    const float al2 = fmaf(dr, dr, dz2);
    const float be2 = fmaf(sr, sr, dz2);
    const float rb = __builtin_amdgcn_rsqf(be2);
    const float m1 = al2 * (rb * rb);
    const float L2 = -__builtin_amdgcn_logf(m1);
    const float K = fmaf(ellipk32_Q(m1), L2, ellipk32_P(m1));
    const float E = fmaf(ellipe32_Q(m1), L2, ellipe32_P(m1));
    const float f = sv * rb * __builtin_amdgcn_rcpf(al2);
    const float alK = al2 * K;
    const float gz = fmaf(fmaf(-dr, sr, -dz2), E, alK);
    const float gr = dz * fmaf(0.5f * (al2 + be2), E, -alK);
    az = fmaf(f, gz, az);
    ar = fmaf(f, gr, ar);
}

// Can a pair of 64-element groups with these grid bounding boxes reach
// m1 < m1_near?  m1 >= min al2 / max be2 over the boxes.
__device__ __forceinline__ bool groups_near(int4 a, int4 b, float c2f, float m1_near) {
    const int dr = max(0, max(b.x - a.y, a.x - b.y));
    const int dz = max(0, max(b.z - a.w, a.z - b.w));
    const float al2 = (float)(dr * dr + dz * dz);
    const float sr = c2f + (float)(a.y + b.y);
    const int dzm = max(abs(a.w - b.z), abs(b.w - a.z));
    const float be2 = fmaf(sr, sr, (float)dzm * (float)dzm);
    return al2 < m1_near * be2 * 1.0001f;
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Transposed pairs: contribution of target e (weights wr, wz) to the
// unit-strength source j: wr * g_r(e, j) + wz * g_z(e, j).  (dr, dz, sr) are the
// target-minus-source offsets and radius sum, as in pair64 / pair32.
__device__ __forceinline__ void pairT64(double dr, double dz, double sr, double wr, double wz,
                                        double &acc) {
    const double dz2 = dz * dz;
    const double al2 = fma(dr, dr, dz2);
    const double be2 = fma(sr, sr, dz2);
    const double rb = rsqrt(be2);
    const double m1 = al2 * (rb * rb);
    const double L = -log(m1);
    const double K = fma(ellipk64_Q(m1), L, ellipk64_P(m1));
    const double E = fma(ellipe64_Q(m1), L, ellipe64_P(m1));
    const double f = rb / al2;
    const double alK = al2 * K;
    const double gz = fma(fma(-dr, sr, -dz2), E, alK);
    const double gr = dz * fma(0.5 * (al2 + be2), E, -alK);
    const bool ok = al2 > 0.0;
    acc = ok ? fma(f, fma(wr, gr, wz * gz), acc) : acc;
}

__device__ __forceinline__ void pairT32(float dr, float dz, float sr, float wr, float wz, float &acc) {
    const float dz2 = dz * dz;
    const float al2 = fmaf(dr, dr, dz2);
    const float be2 = fmaf(sr, sr, dz2);
    const float rb = __builtin_amdgcn_rsqf(be2);
    const float m1 = al2 * (rb * rb);
    const float L2 = -__builtin_amdgcn_logf(m1);
    const float K = fmaf(ellipk32_Q(m1), L2, ellipk32_P(m1));
    const float E = fmaf(ellipe32_Q(m1), L2, ellipe32_P(m1));
    const float f = rb * __builtin_amdgcn_rcpf(al2);
    const float alK = al2 * K;
    const float gz = fmaf(fmaf(-dr, sr, -dz2), E, alK);
    const float gr = dz * fmaf(0.5f * (al2 + be2), E, -alK);
    acc = fmaf(f, fmaf(wr, gr, wz * gz), acc);
}

__device__ __forceinline__ double T_of_u(const RunConst &rc, double u) {
    const double x = fma(u, rc.u_a1, rc.u_a0);
    return rc.T_ref * (rc.cp_exp == 3.0 ? sqrt(sqrt(x)) : pow(x, rc.u_inv));
}

// Local law at step k: Jc(B, T, eps) and E, dE/dJ.  Power law
// E = Ec x^n sgn J, x = |J|/Jc.  With rho_n > 0 the power-law resistivity
// p = E/J = (Ec/Jc) x^(n-1) acts in parallel with rho_n (flux creep, flux flow
// and normal state in one law): E = rho_n p/(p + rho_n) J and
// dE/dJ = rho_n p/(p + rho_n) (n rho_n + p)/(rho_n + p); Jc <= 0, or p beyond
// FP64 range, is the normal state E = rho_n J.  Returns the status bits
// (ST_JC when the pure power law meets J != 0 with Jc <= 0).
struct Local {
    double Jc, x, E, Ep, fT, fB, Bm, p;
};
__device__ __forceinline__ unsigned local_law(const RunConst &rc, double cw, double jcs, double J,
                                              double T, double br, double bz, Local &o) {
    o.Bm = sqrt(br * br + bz * bz);
    o.fT = fmax(0.0, 1.0 - T / rc.Tc);
    o.fB = rc.B0 / (rc.B0 + o.Bm);
    o.Jc = cw * jcs * o.fT * o.fB;
    o.E = 0.0;
    o.Ep = 0.0;
    o.x = 0.0;
    o.p = 0.0;
    if (rc.rho_n > 0.0 && !(o.Jc > 0.0)) {  // normal state
        o.E = rc.rho_n * J;
        o.Ep = rc.rho_n;
        o.x = J != 0.0 ? INFINITY : 0.0;
        o.p = INFINITY;
        return 0u;
    }
    if (J == 0.0) return 0u;
    if (!(o.Jc > 0.0)) return ST_JC;
    o.x = fabs(J) / o.Jc;
    const double p = pow(o.x, rc.n - 1.0);
    if (rc.rho_n > 0.0) {
        const double rn = rc.rho_n;
        o.p = rc.Ec / o.Jc * p;
        if (!isfinite(o.p)) {
            o.E = rn * J;
            o.Ep = rn;
            return 0u;
        }
        const double sfr = o.p / (o.p + rn);
        o.E = rn * sfr * J;
        o.Ep = rn * sfr * ((rc.n * rn + o.p) / (rn + o.p));
        return 0u;
    }
    o.Ep = rc.n * rc.Ec / o.Jc * p;
    o.E = copysign(rc.Ec * p * o.x, J);
    return 0u;
}

// Adjoint of the local law: given Eb = dObj/dE and Epb = dObj/dE' at current
// density J, the derivatives with respect to J (Jc held) and to Jc (J held).
// Zero-measure kinks (J = 0) take the zero branch.
__device__ __forceinline__ void local_law_adj(const RunConst &rc, const Local &lo, double J, double Eb,
                                              double Epb, double &Jb, double &Jcb) {
    Jb = 0.0;
    Jcb = 0.0;
    if (rc.rho_n > 0.0 && (!(lo.Jc > 0.0) || !isfinite(lo.p))) {  // normal state: E = rho_n J
        Jb = Eb * rc.rho_n;
        return;
    }
    if (J == 0.0 || !(lo.Jc > 0.0)) return;
    if (rc.rho_n > 0.0) {
        // p = Ec |J|^(n-1) / Jc^n; E = rho_n s J, E' = rho_n s t with
        // s = p/(p + rho_n), t = (n rho_n + p)/(rho_n + p)
        const double rn = rc.rho_n, n = rc.n, p = lo.p;
        const double den = p + rn;
        const double sfr = p / den, tfr = (n * rn + p) / den;
        const double ds = rn / (den * den), dtt = (1.0 - n) * rn / (den * den);
        const double dEp_dp = rn * (ds * tfr + sfr * dtt);
        const double dp_dJ = (n - 1.0) * p / J, dp_dJc = -n * p / lo.Jc;
        Jb = Eb * lo.Ep + Epb * dEp_dp * dp_dJ;
        Jcb = Eb * rn * J * ds * dp_dJc + Epb * dEp_dp * dp_dJc;
        return;
    }
    // E = Ec x^n sgn J, E' = n Ec x^(n-1) / Jc, x = |J| / Jc
    const double x = lo.x, sg = J > 0.0 ? 1.0 : -1.0;
    const double xn2 = pow(x, rc.n - 2.0);
    const double xb = Eb * rc.Ec * rc.n * xn2 * x * sg + Epb * rc.n * rc.Ec * (rc.n - 1.0) * xn2 / lo.Jc;
    Jcb = -Epb * lo.Ep / lo.Jc - xb * x / lo.Jc;
    Jb = xb * sg / lo.Jc;
}

// v of lane j (j uniform) to every lane, by two scalar reads
__device__ __forceinline__ double lane_value(double v, int j) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), j);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Symmetric n x n matrices in LDS are kept as their lower triangle, packed
// by columns: entry (i, j), i >= j, at pcol(n, j) + i - j; n (n + 1) / 2
// doubles (16.25 KiB at n = 64, so that nine wires' workgroups share a CU).
// Consecutive rows of a column are consecutive in LDS (no bank conflicts when
// lane i reads row i), a row's entries are at varying strides.
__device__ __forceinline__ int pcol(int n, int j) { return j * n - ((j * (j - 1)) >> 1); }

// Cholesky of the packed n x n matrix in LDS, one wavefront, one row per lane;
// lower factor in place.  `dummy` is kCholPad doubles of LDS next to it: lanes
// with nothing to store write there instead of branching around the store.
// The trailing update of column j reads eight columns' entries before it
// writes any of them back (their loads are in flight together, where one
// read-modify-write per column would wait out the LDS latency each time);
// every entry gets the same single FMA as in a column-by-column update.
__device__ __forceinline__ unsigned chol_lds(double *sm, int n, int lane, bool act, double *dummy) {
    unsigned bad = 0;
    for (int j = 0; j < n; ++j) {
        const int cj = pcol(n, j);
        __syncthreads();
        const double djj = sm[cj];
        if (!(djj > 0.0)) bad |= ST_PIVOT;
        const double ljj = sqrt(djj);
        __syncthreads();
        // column j scaled by its pivot (rows j .. n - 1)
        const bool inj = act && lane >= j;
        const int aj = inj ? cj + lane - j : 0;
        const double cv = sm[aj];
        const double lv = (lane == j) ? ljj : cv / ljj;
        *(inj ? sm + aj : dummy + lane) = lv;
        __syncthreads();
        const double lij = (act && lane > j) ? lv : 0.0;
        int k0 = j + 1;
        for (; k0 + 8 <= n; k0 += 8) {
            // eight whole columns k0 .. k0 + 7: column k0 + q starts at
            // pcol(n, k0) + q (n - k0) - q (q - 1) / 2, so the addresses are one
            // scalar base plus compile-time multiples (the general form below
            // costs a dozen scalar instructions per column); lanes above a
            // column's diagonal read an in-range entry they do not use
            const int base = pcol(n, k0) - k0 + lane, st1 = n - k0 - 1;
            double lk[8], ak[8];
            int addr[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                lk[q] = sm[cj + k0 + q - j];
                addr[q] = act ? base + q * st1 - ((q * (q - 1)) >> 1) : 0;
                ak[q] = sm[addr[q]];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool st = act && lane >= k0 + q;
                *(st ? sm + addr[q] : dummy + lane) = ak[q] - lij * lk[q];
            }
        }
        if (k0 < n) {
            // the last, partial chunk: columns k0 .. k0 + nq - 1, the same
            // addressing with the padding slots q >= nq reading column
            // k0 + nq - 1 (in range, not stored)
            const int nq = n - k0;
            const int base = pcol(n, k0) - k0 + lane, st1 = n - k0 - 1;
            double lk[8], ak[8];
            int addr[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int qq = q < nq ? q : nq - 1;
                lk[q] = sm[cj + k0 + qq - j];
                addr[q] = act ? base + qq * st1 - ((qq * (qq - 1)) >> 1) : 0;
                ak[q] = sm[addr[q]];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool st = act && q < nq && lane >= k0 + q;
                *(st ? sm + addr[q] : dummy + lane) = ak[q] - lij * lk[q];
            }
        }
    }
    __syncthreads();
    return bad;
}

// Solve L L^T v_q = v_q for K right-hand sides at once (packed factor in LDS,
// lane i holding entry i of every v_q).  v_j comes from lane j by scalar
// reads, and so does 1 / L_jj: every lane forms the reciprocal of its own
// pivot once, in parallel, so that the chain from one j to the next holds a
// multiplication rather than a division (the same values as a division per
// step); the factor's entries of the next j are read while the current j is
// applied.
template <int K>
__device__ __forceinline__ void solve_lds(const double *sm, int n, int lane, bool act, double (&v)[K]) {
    const double rp = act ? 1.0 / sm[pcol(n, lane)] : 1.0;
    double l = (act && lane > 0) ? sm[lane] : 0.0;
    int cn = 0;  // pcol(n, j + 1), advanced by n - j per step
    for (int j = 0; j < n; ++j) {
        const int jn = j + 1 < n ? j + 1 : j;
        cn += j + 1 < n ? n - j : 0;
        const double l_n = (act && lane > jn) ? sm[cn + lane - jn] : 0.0;
        const double rjj = lane_value(rp, j);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double vj = lane_value(v[q], j) * rjj;
            if (lane == j) v[q] = vj;
            if (act && lane > j) v[q] -= l * vj;
        }
        l = l_n;
    }
    // backward: lane i < j needs L(j, i), row j of the factor
    l = (act && lane < n - 1) ? sm[pcol(n, lane) + n - 1 - lane] : 0.0;
    for (int j = n - 1; j >= 0; --j) {
        const int jn = j > 0 ? j - 1 : 0;
        const double l_n = (act && lane < jn) ? sm[pcol(n, lane) + jn - lane] : 0.0;
        const double rjj = lane_value(rp, j);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double vj = lane_value(v[q], j) * rjj;
            if (lane == j) v[q] = vj;
            if (act && lane < j) v[q] -= l * vj;
        }
        l = l_n;
    }
}

// The factor again, packed by rows: entry (i, j), j <= i, at prow(i) + j, so
// that the backward sweep's reads of row j are consecutive in LDS (by
// columns they are n - i apart: bank conflicts once per column step).  Worth
// its LDS where one factor serves many solves.
__device__ __forceinline__ int prow(int i) { return (i * (i + 1)) >> 1; }

__device__ __forceinline__ void factor_rows_lds(const double *Lc, double *Lr, int n, int lane, bool act) {
    for (int j = 0; j < n; ++j)
        if (act && lane >= j) Lr[prow(lane) + j] = Lc[pcol(n, j) + lane - j];
    __syncthreads();
}

// solve_lds with the backward sweep on the row copy Lr (same arithmetic)
template <int K>
__device__ __forceinline__ void solve_lds_rows(const double *sm, const double *Lr, int n, int lane, bool act,
                                               double (&v)[K]) {
    const double rp = act ? 1.0 / sm[pcol(n, lane)] : 1.0;
    double l = (act && lane > 0) ? sm[lane] : 0.0;
    int cn = 0;  // pcol(n, j + 1), advanced by n - j per step
    for (int j = 0; j < n; ++j) {
        const int jn = j + 1 < n ? j + 1 : j;
        cn += j + 1 < n ? n - j : 0;
        const double l_n = (act && lane > jn) ? sm[cn + lane - jn] : 0.0;
        const double rjj = lane_value(rp, j);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double vj = lane_value(v[q], j) * rjj;
            if (lane == j) v[q] = vj;
            if (act && lane > j) v[q] -= l * vj;
        }
        l = l_n;
    }
    l = (act && lane < n - 1) ? Lr[prow(n - 1) + lane] : 0.0;
    for (int j = n - 1; j >= 0; --j) {
        const int jn = j > 0 ? j - 1 : 0;
        const int rn = prow(jn);
        const double l_n = (act && lane < jn) ? Lr[rn + lane] : 0.0;
        const double rjj = lane_value(rp, j);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double vj = lane_value(v[q], j) * rjj;
            if (lane == j) v[q] = vj;
            if (act && lane < j) v[q] -= l * vj;
        }
        l = l_n;
    }
}

// Solve L L^T [x y] = [x y] with the packed factor in LDS; lane i holds entry i.
__device__ __forceinline__ void solve2_lds(const double *sm, int n, int lane, bool act, double &xv, double &yv) {
    double v[2] = {xv, yv};
    solve_lds<2>(sm, n, lane, act, v);
    xv = v[0];
    yv = v[1];
}

// Load the lower triangle of the layer's inductance block (column-major
// n x n in global memory) into packed LDS and add dt diag(2 pi r E'/d^2).
__device__ __forceinline__ void load_wire_matrix(double *sm, const double *M, int n, int lane, bool act,
                                                 double diag_add) {
    // 16 column loads in flight; every active lane loads (the entries above
    // the diagonal are not kept), and lanes with nothing to keep store to the
    // sink after the packed matrix, so no load or store sits under a branch
    double *sink = sm + packed_size(n) + lane;
    if (act)
        for (int c0 = 0; c0 < n; c0 += 16) {
            double a[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) a[q] = c0 + q < n ? M[(size_t)(c0 + q) * n + lane] : 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int c = c0 + q;
                *(c < n && lane >= c ? sm + pcol(n, c) + lane - c : sink) = a[q];
            }
        }
    __syncthreads();
    if (act) sm[pcol(n, lane)] += diag_add;
}

// y_i = sum_j A_ij v_j with the column-major n x n block in LDS (lane i
// holding row i), v_j from lane j, the FMAs in j order.  Eight LDS reads are
// issued before their FMAs, and no read sits under a branch (lanes past n
// read row 0 and return 0).
__device__ __forceinline__ double matvec_lds(const double *A, int n, bool act, int lane, double v) {
    double y = 0.0;
    const int li = act ? lane : 0;
    for (int j0 = 0; j0 < n; j0 += 8) {
        double a[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = j0 + q < n ? A[(j0 + q) * n + li] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (j0 + q < n) y = fma(a[q], lane_value(v, j0 + q), y);
    }
    return act ? y : 0.0;
}

__device__ __forceinline__ double matvec_cols(const double *A, int n, int lane, bool act, double v) {
    double y = 0.0;
    for (int j0 = 0; j0 < n; j0 += 16) {
        double a[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) a[q] = (act && j0 + q < n) ? A[(size_t)(j0 + q) * n + lane] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (j0 + q < n) {
                const double vj = __shfl(v, j0 + q);
                if (act) y = fma(a[q], vj, y);
            }
    }
    return y;
}

}  // namespace coilq
