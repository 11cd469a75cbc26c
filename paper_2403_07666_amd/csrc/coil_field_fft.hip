// coil_field_fft.hip -- field pass by fast convolution along z (the layout,
// the spectra and the three steps of a pass are described in coil_field_fft.h).
//
// Layouts (per coil, rows padded to Rp):
//   spectra   G^_z[f][j][i], then S[f][j][i]  (j source row, i target row), TS reals:
//             FP32 in mixed precision (the only data a pass streams from HBM), else FP64.
//             S is symmetric (g_r depends on the two rows through (i - j)^2 and i + j
//             only), so in FP64 a coil of one block (n_r <= 256) keeps per bin only
//             its upper triangle packed by rows (sym_row): 3/4 of the bytes per pass
//   hat       FP64; forward: I^[f][j] (re, im); transposed: W^[f][i] (wr re, wr im, wz re, wz im)
//   bpart     FP64; forward: [p][i][f] (Bz^ re, Bz^ im, Br^ re, Br^ im), p = source-row part;
//             transposed: [ib][j][f] (re, im), ib = target block.  Bin-minor, so that
//             the inverse DFT of a row reads its bins contiguously; the bin products
//             write them scattered (a small share of their traffic)
// The DFTs run in FP64 (radix-2, decimation in time, in LDS, one row or two
// real rows packed as one complex row per workgroup), and so do the bin
// products' sums: in mixed precision only the stored spectra are rounded (to
// FP32, a relative 2^-24 per value), which keeps the pass's error at about
// that of the rounded kernel values.  The DFT's own FP32 rounding would be
// relative to the norm of the whole row instead, and a row packs B_z with the
// smaller B_r.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "coil_device.h"
#include "coil_field_fft.h"

namespace coilq {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
// 4 consecutive reals as doubles (16-byte aligned for float, 32 for double)
__device__ __forceinline__ void load4(const float *p, double (&v)[4]) {
    const f4v q = *reinterpret_cast<const f4v *>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
}
__device__ __forceinline__ void load4(const double *p, double (&v)[4]) {
    const d2v a = reinterpret_cast<const d2v *>(p)[0];
    const d2v b = reinterpret_cast<const d2v *>(p)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}
__device__ __forceinline__ void store4(double *p, double a, double b, double c, double d) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(a, b);
    reinterpret_cast<double2 *>(p)[1] = make_double2(c, d);
}

// Four consecutive reals of one source row as loaded (converted to FP64 where
// they are used), so that a batch of rows can be in flight before the first
// FMA waits for it.
template <typename TS>
struct Row4;
template <>
struct Row4<float> {
    f4v v;
    __device__ __forceinline__ void ld(const float *p) { v = *reinterpret_cast<const f4v *>(p); }
    __device__ __forceinline__ double operator[](int t) const { return (double)v[t]; }
};
template <>
struct Row4<double> {
    d2v a, b;
    __device__ __forceinline__ void ld(const double *p) {
        a = reinterpret_cast<const d2v *>(p)[0];
        b = reinterpret_cast<const d2v *>(p)[1];
    }
    __device__ __forceinline__ double operator[](int t) const { return t < 2 ? a[t] : b[t - 2]; }
};

// waves per bin-product workgroup (they split the workgroup's source rows;
// eight measured 4-10 % slower than four)
constexpr int kFftW = 4;
// source rows per batch of the FP32 bin products (two batches in flight per
// wave; FP64 spectra: half as many rows).  Eight measured the same, and
// bounding the kernel to three waves per SIMD (which spills) 1-2 % slower.
constexpr int kFftNB = 4;
// rows per group of the symmetric kernels' double-buffered loops (four: 320
// VGPRs, one wave per SIMD, 3 % slower than two)
constexpr int kFftSG = 2;

__device__ __forceinline__ int bitrev(int m, int logL) {
    return (int)(__builtin_bitreverse32((unsigned)m) >> (32 - logL));
}

// In-place DFT X[f] = sum_m x[m] exp(-2 pi i f m / L) of the L values in a[]
// (LDS), stored by the caller in bit-reversed order (then a barrier); the
// result is in natural order, followed by a barrier.  Radix-2 stage s
// combines pairs half = 2^(s-1) apart with the twiddle W_{2 half}^pos =
// exp(-2 pi i pos / 2^s), read from the table of exp(-2 pi i k / Lmax) at
// k = pos Lmax / 2^s.  Two stages at a time (radix 2^2): a thread takes the
// four values pos + {0, 1, 2, 3} half of a group of 4 half, applies stage s to
// the pairs (0, 1), (2, 3) and stage s + 1 to (0, 2) with W_{4 half}^pos and
// (1, 3) with W_{4 half}^(pos + half) = -i W_{4 half}^pos, in registers; one
// LDS round trip and barrier per two stages, a last radix-2 stage if log2 L
// is odd.
__device__ __forceinline__ double2 cmul(double2 w, double2 v) {
    return make_double2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
}

__device__ void fft_lds(double2 *a, int L, int logL, const double2 *__restrict__ tw, int logLmax) {
    int s = 1;
    for (; s + 1 <= logL; s += 2) {
        const int half = 1 << (s - 1);
        for (int k = threadIdx.x; k < (L >> 2); k += blockDim.x) {
            const int pos = k & (half - 1);
            const int i0 = ((k >> (s - 1)) << (s + 1)) | pos;
            const double2 a0 = a[i0], a1 = a[i0 + half], a2 = a[i0 + 2 * half], a3 = a[i0 + 3 * half];
            const double2 w1 = tw[pos << (logLmax - s)];
            const double2 w2 = tw[pos << (logLmax - s - 1)];
            const double2 t1 = cmul(w1, a1), t3 = cmul(w1, a3);
            const double2 b0 = make_double2(a0.x + t1.x, a0.y + t1.y), b1 = make_double2(a0.x - t1.x, a0.y - t1.y);
            const double2 b2 = make_double2(a2.x + t3.x, a2.y + t3.y), b3 = make_double2(a2.x - t3.x, a2.y - t3.y);
            const double2 u = cmul(w2, b2), v0 = cmul(w2, b3);
            const double2 v = make_double2(v0.y, -v0.x);  // -i w2 b3
            a[i0] = make_double2(b0.x + u.x, b0.y + u.y);
            a[i0 + 2 * half] = make_double2(b0.x - u.x, b0.y - u.y);
            a[i0 + half] = make_double2(b1.x + v.x, b1.y + v.y);
            a[i0 + 3 * half] = make_double2(b1.x - v.x, b1.y - v.y);
        }
        __syncthreads();
    }
    if (s == logL) {
        const int half = 1 << (s - 1);
        for (int k = threadIdx.x; k < (L >> 1); k += blockDim.x) {
            const int pos = k & (half - 1);
            const int i0 = ((k >> (s - 1)) << s) | pos;
            const double2 t = cmul(tw[pos << (logLmax - s)], a[i0 + half]);
            const double2 u = a[i0];
            a[i0] = make_double2(u.x + t.x, u.y + t.y);
            a[i0 + half] = make_double2(u.x - t.x, u.y - t.y);
        }
        __syncthreads();
    }
}

// Inverse transform of two real rows u, v from their half spectra U, V
// (bins f = 0 .. L/2; get(f) returns (U re, U im, V re, V im)): the row
// y = u + i v has the spectrum Y = U + i V, with Y[L - f] = conj(U[f]) +
// i conj(V[f]); y = conj(DFT(conj Y)) / L.  Leaves DFT(conj Y) in a[].
template <typename Get>
__device__ __forceinline__ void inverse_pair(double2 *a, const FftCoil &C, const FftPlan &fp, Get get) {
    const int L = C.L, logL = C.logL, half = L >> 1;
    for (int f = threadIdx.x; f < C.bins; f += blockDim.x) {
        double ur, ui, vr, vi;
        get(f, ur, ui, vr, vi);
        a[bitrev(f, logL)] = make_double2(ur - vi, -(ui + vr));
        if (f > 0 && f < half) a[bitrev(L - f, logL)] = make_double2(ur + vi, ui - vr);
    }
    __syncthreads();
    fft_lds(a, L, logL, fp.tw64, fp.logLmax);
}

// ------------------------------------------------------------------ set-up
// Mutual inductance of two coaxial rings over mu0 d (Maxwell's formula with
// the modulus m1 = al^2 / be^2 of the field kernel, grid units), zero for the
// element's own ring; even in dz.
__device__ __forceinline__ double flux_kernel(double dr, double dz, double sr) {
    const double dz2 = dz * dz;
    const double al2 = fma(dr, dr, dz2);
    const double be2 = fma(sr, sr, dz2);
    if (!(al2 > 0.0)) return 0.0;
    const double rb = rsqrt(be2);
    const double m1 = al2 * (rb * rb);
    const double L = -log(m1);
    const double K = fma(ellipk64_Q(m1), L, ellipk64_P(m1));
    const double E = fma(ellipe64_Q(m1), L, ellipe64_P(m1));
    return sqrt(be2) * fma(0.5 * (1.0 + m1), K, -E);
}

// One workgroup per (target row a, source row b of the slab): the FP64 kernel
// values g(a - b, delta) for delta = 0 .. Z-1, placed at m = delta and (their
// mirrors: g_z even, g_r odd) at m = L - delta as x = g_z + i g_r, the DFT,
// and per bin G^_z = (X[f] + X[L-f]) / 2, S = (X[L-f] - X[f]) / 2 (real parts).
// kind 1: the flux kernel (even, real spectrum M^ = Re X[f]) in the first place.
__global__ __launch_bounds__(256) void k_fft_spec(FftPlan fp, int coil, int b0, double2 *tmp, int kind) {
    extern __shared__ double2 xs[];
    const FftCoil C = fp.coils[coil];
    const int a = blockIdx.x, bl = blockIdx.y, b = b0 + bl;
    const int L = C.L, logL = C.logL;
    for (int m = threadIdx.x; m < L; m += blockDim.x) xs[m] = make_double2(0.0, 0.0);
    __syncthreads();
    const double dr = (double)(a - b), sr = C.c2d + (double)(a + b);
    for (int d = threadIdx.x; d < C.Z; d += blockDim.x) {
        double gr = 0.0, gz = 0.0;
        if (kind == 1)
            gz = flux_kernel(dr, (double)d, sr);
        else
            pair64(dr, (double)d, sr, 1.0, gr, gz);  // zero for the element's own ring
        xs[bitrev(d, logL)] = make_double2(gz, gr);
        if (d > 0) xs[bitrev(L - d, logL)] = make_double2(gz, -gr);
    }
    __syncthreads();
    fft_lds(xs, L, logL, fp.tw64, fp.logLmax);
    double2 *out = tmp + ((size_t)bl * C.R + a) * C.bins;
    for (int f = threadIdx.x; f < C.bins; f += blockDim.x) {
        const double2 X = xs[f], Y = xs[(L - f) & (L - 1)];
        out[f] = make_double2(0.5 * (X.x + Y.x), 0.5 * (Y.x - X.x));
    }
}

// the slab's spectra from [b][a][f] to [f][b][a] (a < Rp; zeros past R), as T,
// into dst: the first place, and the second a plane (bins R Rp) later if
// planes = 2 -- packed by rows (a <= b, zeros up to the row's padded length)
// for a coil with sym
template <typename T>
__global__ __launch_bounds__(256) void k_fft_spec_store(FftPlan fp, int coil, int b0, const double2 *tmp, T *dst,
                                                        int planes) {
    __shared__ double2 tile[32][33];
    const FftCoil C = fp.coils[coil];
    const int f0 = blockIdx.x * 32, a0 = blockIdx.y * 32, bl = blockIdx.z, b = b0 + bl;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = 0; k < 32; k += 8) {
        const int a = a0 + ty + k, f = f0 + tx;
        tile[ty + k][tx] =
            (a < C.R && f < C.bins) ? tmp[((size_t)bl * C.R + a) * C.bins + f] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    T *gz = dst;
    T *gs = gz + (size_t)C.bins * C.R * C.Rp;
    for (int k = 0; k < 32; k += 8) {
        const int f = f0 + ty + k, a = a0 + tx;
        if (f < C.bins && a < C.Rp) {
            const double2 v = tile[tx][ty + k];
            const size_t o = ((size_t)f * C.R + b) * C.Rp + a;
            gz[o] = (T)v.x;
            if (planes == 2 && !C.sym) gs[o] = (T)v.y;
            if (planes == 2 && C.sym && a < 4 * ((b >> 2) + 1))
                gs[(size_t)f * C.sp + sym_row(b) + a] = a <= b ? (T)v.y : (T)0;
        }
    }
}

// ------------------------------------------------------------------ forward pass
// source rows a = 2q, b = 2q + 1 as one complex row k (I_a + i I_b) (k the
// field's kscale, or the flux kernel's mu0 d), zero-padded to L;
// I^_a = (X[f] + conj X[L-f]) / 2, I^_b = (X[f] - conj X[L-f]) / 2i
__global__ __launch_bounds__(256) void k_fft_rows_fwd(FftPlan fp, const double *__restrict__ I,
                                                      const int *__restrict__ pub2int, int kind,
                                                      const int *__restrict__ done) {
    extern __shared__ double2 xs[];
    if (done && *done) return;
    const int4 it = fp.items[blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const double k = kind == 1 ? C.kflux : C.kscale;
    const int a = 2 * it.y, b = a + 1;
    const int L = C.L, logL = C.logL, Z = C.Z;
    const bool hb = b < C.R;
    const int *pa = pub2int + C.off + (size_t)a * Z;
    for (int z = threadIdx.x; z < L; z += blockDim.x) {
        double va = 0.0, vb = 0.0;
        if (z < Z) {
            va = k * I[pa[z]];
            if (hb) vb = k * I[pa[Z + z]];
        }
        xs[bitrev(z, logL)] = make_double2(va, vb);
    }
    __syncthreads();
    fft_lds(xs, L, logL, fp.tw64, fp.logLmax);
    double *hat = fp.hat + C.hat;
    for (int f = threadIdx.x; f < C.bins; f += blockDim.x) {
        const double2 X = xs[f], Y = xs[(L - f) & (L - 1)];
        const size_t o = ((size_t)f * C.R + a) * 2;
        hat[o] = 0.5 * (X.x + Y.x);
        hat[o + 1] = 0.5 * (X.y - Y.y);
        if (hb) {
            hat[o + 2] = 0.5 * (X.y + Y.y);
            hat[o + 3] = 0.5 * (Y.x - X.x);
        }
    }
}

// Bin products, one workgroup per (coil, bin f, block of kFftI targets, part of
// kFftJ sources): Bz^_i = sum_j G^_z,ij I^_j, Br^_i = i sum_j S_ij I^_j.  A lane
// owns 4 consecutive targets (one 16/32-byte load per matrix and source row),
// the four waves split the part's sources and add in LDS in a fixed order.
// TS: the stored spectra (the sums are FP64).  FLUX: the one real matrix M^ of
// the flux kernel (FP64) in place of (G^_z, S), its product in the B_z places.
template <typename TS, int FLUX>
__global__ __launch_bounds__(64 * kFftW) void k_fft_bins(FftPlan fp, const int4 *__restrict__ items,
                                                        const int *__restrict__ done) {
    __shared__ double2 sI[kFftJ];
    __shared__ double red[kFftW - 1][16][65];
    if (done && *done) return;
    const int4 it = items[blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const int f = it.y, j0 = it.w * kFftJ;
    const int jn = min(kFftJ, C.R - j0);
    const double *hat = fp.hat + C.hat;
    if ((int)threadIdx.x < jn) {
        const size_t o = ((size_t)f * C.R + j0 + threadIdx.x) * 2;
        sI[threadIdx.x] = make_double2(hat[o], hat[o + 1]);
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = it.z * kFftI + 4 * lane;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    constexpr int JW = kFftJ / kFftW;
    const int jw0 = w * JW, jw1 = min(jw0 + JW, jn);
    // Rows in batches of NB, two batches in registers: the loads of the next
    // batch are issued before the FMAs of the current one, so that two batches
    // of each wave stay in flight; the FMAs of each sum in ascending j as in a
    // plain loop.
    constexpr int NB = (sizeof(TS) == 4 || FLUX) ? kFftNB : kFftNB / 2;
    const int nfull = jw1 > jw0 ? (jw1 - jw0) / NB : 0;
    if (i < C.Rp) {
        const size_t plane = (size_t)C.bins * C.R * C.Rp;
        const TS *gz = FLUX ? reinterpret_cast<const TS *>(fp.fspec + C.fspec)
                            : static_cast<const TS *>(fp.spec) + C.spec;
        gz += ((size_t)f * C.R + j0) * C.Rp + i;
        Row4<TS> ga[NB], sa[NB], gb[NB], sb[NB];
        auto load = [&](Row4<TS>(&g)[NB], Row4<TS>(&sv)[NB], int j) {
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                g[u].ld(gz + (size_t)(j + u) * C.Rp);
                if (!FLUX) sv[u].ld(gz + plane + (size_t)(j + u) * C.Rp);
            }
        };
        auto fmas = [&](const Row4<TS> &g, const Row4<TS> &sv, double2 x) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                acc[t] = fma(g[t], x.x, acc[t]);
                acc[4 + t] = fma(g[t], x.y, acc[4 + t]);
                if (!FLUX) {
                    acc[8 + t] = fma(-sv[t], x.y, acc[8 + t]);
                    acc[12 + t] = fma(sv[t], x.x, acc[12 + t]);
                }
            }
        };
        auto comp = [&](const Row4<TS>(&g)[NB], const Row4<TS>(&sv)[NB], int j) {
            // the scheduler would otherwise sink the loads issued just before
            // below these FMAs (it trades their latency for registers)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < NB; ++u) fmas(g[u], sv[u], sI[j + u]);
        };
        // (the loop body has no branch and the prefetch of its second batch is
        // clamped -- past the last batch it re-reads it -- so that no load sits
        // in a branch between its issue and the FMAs of an earlier batch, which
        // would make those wait for it)
        if (nfull > 0) {
            load(ga, sa, jw0);
            for (int k = 0; k + 1 < nfull; k += 2) {
                load(gb, sb, jw0 + (k + 1) * NB);
                comp(ga, sa, jw0 + k * NB);
                load(ga, sa, jw0 + min(k + 2, nfull - 1) * NB);
                comp(gb, sb, jw0 + (k + 1) * NB);
            }
            if (nfull & 1) comp(ga, sa, jw0 + (nfull - 1) * NB);
        }
        for (int j = jw0 + nfull * NB; j < jw1; ++j) {
            ga[0].ld(gz + (size_t)j * C.Rp);
            if (!FLUX) sa[0].ld(gz + plane + (size_t)j * C.Rp);
            fmas(ga[0], sa[0], sI[j]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) red[w - 1][q][lane] = acc[q];
    }
    __syncthreads();
    if (w == 0 && i < C.Rp) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            for (int v = 0; v < kFftW - 1; ++v) acc[q] += red[v][q][lane];
        double *out = fp.bpart + C.bpart + (((size_t)it.w * C.Rp + i) * C.bins + f) * 4;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            store4(out + (size_t)t * C.bins * 4, acc[t], acc[4 + t], acc[8 + t], acc[12 + t]);
    }
}

// target row i: Y = Bz^ + i Br^ (the parts summed in order), inverse DFT,
// part[0][e] = (B_r partial, B_z partial) of the row's elements; kind 1 (the
// flux pass): (0, flux)
__global__ __launch_bounds__(256) void k_fft_rows_inv(FftPlan fp, const int *__restrict__ pub2int,
                                                      double2 *__restrict__ part, int kind,
                                                      const int *__restrict__ done) {
    extern __shared__ double2 xs[];
    if (done && *done) return;
    const int4 it = fp.items[fp.npairs + blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const int i = it.y;
    const double *bp = fp.bpart + C.bpart;
    inverse_pair(xs, C, fp, [&](int f, double &ur, double &ui, double &vr, double &vi) {
        ur = ui = vr = vi = 0.0;
        for (int p = 0; p < C.P; ++p) {
            double v[4];
            load4(bp + (((size_t)p * C.Rp + i) * C.bins + f) * 4, v);
            ur += v[0];
            ui += v[1];
            vr += v[2];
            vi += v[3];
        }
    });
    const double invL = 1.0 / (double)C.L;
    const int *pe = pub2int + C.off + (size_t)i * C.Z;
    for (int z = threadIdx.x; z < C.Z; z += blockDim.x) {
        const double2 F = xs[z];
        part[pe[z]] = make_double2(kind == 1 ? 0.0 : -F.y * invL, F.x * invL);
    }
}

// ------------------------------------------------------------------ transposed pass
// target row i of the weights as one complex row wr + i wz; W^ per bin
__global__ __launch_bounds__(256) void k_fft_rows_fwdT(FftPlan fp, const double *__restrict__ wr,
                                                       const double *__restrict__ wz,
                                                       const int *__restrict__ pub2int) {
    extern __shared__ double2 xs[];
    const int4 it = fp.items[fp.npairs + blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const int i = it.y;
    const int L = C.L, logL = C.logL, Z = C.Z;
    const int *pe = pub2int + C.off + (size_t)i * Z;
    for (int z = threadIdx.x; z < L; z += blockDim.x) {
        double a = 0.0, b = 0.0;
        if (z < Z) {
            const int e = pe[z];
            a = wr[e];
            b = wz[e];
        }
        xs[bitrev(z, logL)] = make_double2(a, b);
    }
    __syncthreads();
    fft_lds(xs, L, logL, fp.tw64, fp.logLmax);
    double *hat = fp.hat + C.hat;
    for (int f = threadIdx.x; f < C.bins; f += blockDim.x) {
        const double2 X = xs[f], Y = xs[(L - f) & (L - 1)];
        store4(hat + ((size_t)f * C.Rp + i) * 4, 0.5 * (X.x + Y.x), 0.5 * (X.y - Y.y), 0.5 * (X.y + Y.y),
               0.5 * (Y.x - X.x));
    }
}


// Transposed bin products, one workgroup per (coil, bin f, kFftJ sources,
// block of kFftI targets): out^_j = sum_i [G^_z,ij W^z_i - i S_ij W^r_i] (the
// transpose takes conj G^).  A lane holds 4 targets' W^; per source row the
// wave adds its 64 lanes.  TS: the stored spectra (the sums are FP64).
template <typename TS>
__global__ __launch_bounds__(256) void k_fft_binsT(FftPlan fp, const int4 *__restrict__ items) {
    const int4 it = items[blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const int f = it.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = it.w * kFftI + 4 * lane;
    const double *hat = fp.hat + C.hat;
    double wrr[4], wri[4], wzr[4], wzi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        wrr[t] = wri[t] = wzr[t] = wzi[t] = 0.0;
        if (i + t < C.R) {
            double v[4];
            load4(hat + ((size_t)f * C.Rp + i + t) * 4, v);
            wrr[t] = v[0];
            wri[t] = v[1];
            wzr[t] = v[2];
            wzi[t] = v[3];
        }
    }
    constexpr int JW = kFftJ / 4;
    const int jw0 = it.z * kFftJ + w * JW, jw1 = min(jw0 + JW, C.R);
    const size_t plane = (size_t)C.bins * C.R * C.Rp;
    const TS *gz = static_cast<const TS *>(fp.spec) + C.spec + (size_t)f * C.R * C.Rp + i;
    double *out = fp.bpart + C.bpart + ((size_t)it.w * C.R * C.bins + f) * 2;
    const bool act = i < C.Rp;
    // double-buffered groups of SG rows with in-bounds loads in place of the
    // branch (a lane past the padded rows has zero weights), as in k_fft_bins
    constexpr int SG = sizeof(TS) == 4 ? kFftNB : kFftNB / 2;
    const int nfull = jw1 > jw0 ? (jw1 - jw0) / SG : 0;
    if (nfull > 0) {
        const TS *gzl = gz + (act ? 0 : C.Rp - 4 - i);
        Row4<TS> ga[SG], sa[SG], gb[SG], sb[SG];
        auto load = [&](Row4<TS>(&g)[SG], Row4<TS>(&sv)[SG], int j0) {
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                g[u].ld(gzl + (size_t)(j0 + u) * C.Rp);
                sv[u].ld(gzl + plane + (size_t)(j0 + u) * C.Rp);
            }
        };
        auto comp = [&](const Row4<TS>(&g)[SG], const Row4<TS>(&sv)[SG], int j0) {
            __builtin_amdgcn_sched_barrier(0);  // keep the loads above (see k_fft_bins)
            double re[SG], im[SG];
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                re[u] = im[u] = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    re[u] = fma(g[u][t], wzr[t], fma(sv[u][t], wri[t], re[u]));
                    im[u] = fma(g[u][t], wzi[t], fma(-sv[u][t], wrr[t], im[u]));
                }
            }
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                re[u] = wave_sum(re[u]);
                im[u] = wave_sum(im[u]);
            }
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < SG; ++u) {
                    out[(size_t)(j0 + u) * C.bins * 2] = re[u];
                    out[(size_t)(j0 + u) * C.bins * 2 + 1] = im[u];
                }
            }
        };
        load(ga, sa, jw0);
        for (int k = 0; k + 1 < nfull; k += 2) {
            load(gb, sb, jw0 + SG * (k + 1));
            comp(ga, sa, jw0 + SG * k);
            load(ga, sa, jw0 + SG * min(k + 2, nfull - 1));
            comp(gb, sb, jw0 + SG * (k + 1));
        }
        if (nfull & 1) comp(ga, sa, jw0 + SG * (nfull - 1));
    }
    int j = jw0 + SG * nfull;
    for (; j + 4 <= jw1; j += 4) {
        double re[4], im[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            re[u] = im[u] = 0.0;
            if (act) {
                double g[4], sv[4];
                load4(gz + (size_t)(j + u) * C.Rp, g);
                load4(gz + plane + (size_t)(j + u) * C.Rp, sv);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    re[u] = fma(g[t], wzr[t], fma(sv[t], wri[t], re[u]));
                    im[u] = fma(g[t], wzi[t], fma(-sv[t], wrr[t], im[u]));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            re[u] = wave_sum(re[u]);
            im[u] = wave_sum(im[u]);
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                out[(size_t)(j + u) * C.bins * 2] = re[u];
                out[(size_t)(j + u) * C.bins * 2 + 1] = im[u];
            }
        }
    }
    for (; j < jw1; ++j) {
        double re = 0.0, im = 0.0;
        if (act) {
            double g[4], sv[4];
            load4(gz + (size_t)j * C.Rp, g);
            load4(gz + plane + (size_t)j * C.Rp, sv);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                re = fma(g[t], wzr[t], fma(sv[t], wri[t], re));
                im = fma(g[t], wzi[t], fma(-sv[t], wrr[t], im));
            }
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            out[(size_t)j * C.bins * 2] = re;
            out[(size_t)j * C.bins * 2 + 1] = im;
        }
    }
}

// Bin products of a coil with sym (n_r <= 256: one workgroup per bin, every
// source row and target).  G^_z as in k_fft_bins.  S from its packed upper
// triangle: stored row j holds S_ij for i <= j, and serves twice -- lane i
// adds S_ij I^_j to its own target i (i <= j; the padding past j holds
// zeros), and the lanes' S_ij I^_i for i < j, summed over the wave, give
// target j's share from the rows above the diagonal.  Wave w takes rows
// 64 w .. 64 w + 63, four at a time.
template <typename TS>
__global__ __launch_bounds__(64 * kFftW) void k_fft_bins_sym(FftPlan fp, const int4 *__restrict__ items) {
    __shared__ double2 sI[kFftI];
    __shared__ double2 tB[kFftI];  // target j's share from row j's stored entries
    __shared__ double red[kFftW - 1][16][65];
    const int4 it = items[blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const int f = it.y, R = C.R;
    const double *hat = fp.hat + C.hat;
    if ((int)threadIdx.x < R) {
        const size_t o = ((size_t)f * R + threadIdx.x) * 2;
        sI[threadIdx.x] = make_double2(hat[o], hat[o + 1]);
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = 4 * lane;
    double2 xi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) xi[t] = i + t < R ? sI[i + t] : make_double2(0.0, 0.0);
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    const bool act = i < C.Rp;
    const TS *gz = static_cast<const TS *>(fp.spec) + C.spec + (size_t)f * R * C.Rp + i;
    const TS *sp = static_cast<const TS *>(fp.spec) + C.spec + (size_t)C.bins * R * C.Rp + (size_t)f * C.sp + i;
    constexpr int JW = kFftI / kFftW;
    const int jw0 = JW * w, jw1 = min(jw0 + JW, R);
    // Whole groups of SG rows, two groups in registers: the loads of the next
    // group are issued before the FMAs and wavefront sums of the current one
    // (as in k_fft_bins); a last partial group as four rows before.  No load sits in a branch: a lane past the padded
    // rows reads the row's last four columns, and a lane past row j's stored
    // part (4 lane > j) its last four entries, both in bounds, and uses zeros
    // in their place -- adding zero products leaves every sum bitwise as if
    // the lane had skipped them.
    constexpr int SG = kFftSG;
    const int nfull = jw1 > jw0 ? (jw1 - jw0) / SG : 0;
    if (nfull > 0) {
        const TS *gzl = gz + (act ? 0 : C.Rp - 4 - i);
        Row4<TS> ga[SG], sa[SG], gb[SG], sb[SG];
        auto load = [&](Row4<TS>(&g)[SG], Row4<TS>(&sv)[SG], int j) {
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                const int jj = j + u, last = 4 * (jj >> 2);
                g[u].ld(gzl + (size_t)jj * C.Rp);
                sv[u].ld(sp - i + sym_row(jj) + min(i, last));
            }
        };
        auto comp = [&](const Row4<TS>(&g)[SG], const Row4<TS>(&sv)[SG], int j) {
            __builtin_amdgcn_sched_barrier(0);  // keep the loads above (see k_fft_bins)
            double pr[SG], pi[SG];
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                const int jj = j + u;
                const double2 x = sI[jj];
                const bool on = lane <= (jj >> 2);
                pr[u] = pi[u] = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    acc[t] = fma(g[u][t], x.x, acc[t]);
                    acc[4 + t] = fma(g[u][t], x.y, acc[4 + t]);
                    const double sv_t = on ? sv[u][t] : 0.0;
                    acc[8 + t] = fma(-sv_t, x.y, acc[8 + t]);
                    acc[12 + t] = fma(sv_t, x.x, acc[12 + t]);
                    const double m = i + t < jj ? sv_t : 0.0;
                    pr[u] = fma(m, xi[t].x, pr[u]);
                    pi[u] = fma(m, xi[t].y, pi[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                pr[u] = wave_sum(pr[u]);
                pi[u] = wave_sum(pi[u]);
            }
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < SG; ++u) tB[j + u] = make_double2(pr[u], pi[u]);
            }
        };
        load(ga, sa, jw0);
        for (int k = 0; k + 1 < nfull; k += 2) {
            load(gb, sb, jw0 + SG * (k + 1));
            comp(ga, sa, jw0 + SG * k);
            load(ga, sa, jw0 + SG * min(k + 2, nfull - 1));
            comp(gb, sb, jw0 + SG * (k + 1));
        }
        if (nfull & 1) comp(ga, sa, jw0 + SG * (nfull - 1));
    }
    for (int j = jw0 + SG * nfull; j < jw1; j += 4) {
        double pr[4], pi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pr[u] = pi[u] = 0.0;
            const int jj = j + u;
            if (jj >= jw1) continue;  // uniform
            const double2 x = sI[jj];
            if (act) {
                double g[4];
                load4(gz + (size_t)jj * C.Rp, g);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    acc[t] = fma(g[t], x.x, acc[t]);
                    acc[4 + t] = fma(g[t], x.y, acc[4 + t]);
                }
            }
            if (lane <= (jj >> 2)) {
                double sv[4];
                load4(sp + sym_row(jj), sv);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    acc[8 + t] = fma(-sv[t], x.y, acc[8 + t]);
                    acc[12 + t] = fma(sv[t], x.x, acc[12 + t]);
                    const double m = i + t < jj ? sv[t] : 0.0;
                    pr[u] = fma(m, xi[t].x, pr[u]);
                    pi[u] = fma(m, xi[t].y, pi[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pr[u] = wave_sum(pr[u]);
            pi[u] = wave_sum(pi[u]);
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j + u < jw1) tB[j + u] = make_double2(pr[u], pi[u]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) red[w - 1][q][lane] = acc[q];
    }
    __syncthreads();
    if (w == 0 && act) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            for (int v = 0; v < kFftW - 1; ++v) acc[q] += red[v][q][lane];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (i + t < R) {  // Br^ += i (the rows-above share)
                acc[8 + t] -= tB[i + t].y;
                acc[12 + t] += tB[i + t].x;
            }
        double *out = fp.bpart + C.bpart + ((size_t)i * C.bins + f) * 4;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            store4(out + (size_t)t * C.bins * 4, acc[t], acc[4 + t], acc[8 + t], acc[12 + t]);
    }
}

// Transposed bin products of a coil with sym: out^_j = sum_i [G^_z,ij W^z_i -
// i S_ij W^r_i].  G^_z and the stored S_ij (i <= j) of row j by a wave sum
// (out_j); the same stored S_ij for i < j also gives out_i its share
// -i S_ij W^r_j, kept in the lane's registers and added once at the end.
template <typename TS>
__global__ __launch_bounds__(64 * kFftW) void k_fft_binsT_sym(FftPlan fp, const int4 *__restrict__ items) {
    __shared__ double2 sW[kFftI];  // W^r of every row
    __shared__ double2 tD[kFftI];  // out^_j from row j's wave sums
    __shared__ double red[kFftW - 1][8][65];
    const int4 it = items[blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const int f = it.y, R = C.R;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = 4 * lane;
    const double *hat = fp.hat + C.hat;
    if ((int)threadIdx.x < R) {
        const double *h4 = hat + ((size_t)f * C.Rp + threadIdx.x) * 4;
        sW[threadIdx.x] = make_double2(h4[0], h4[1]);
    }
    double wrr[4], wri[4], wzr[4], wzi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        wrr[t] = wri[t] = wzr[t] = wzi[t] = 0.0;
        if (i + t < R) {
            double v[4];
            load4(hat + ((size_t)f * C.Rp + i + t) * 4, v);
            wrr[t] = v[0];
            wri[t] = v[1];
            wzr[t] = v[2];
            wzi[t] = v[3];
        }
    }
    __syncthreads();
    double ar[4], ai[4];  // the lane's outputs' shares from rows below
#pragma unroll
    for (int t = 0; t < 4; ++t) ar[t] = ai[t] = 0.0;
    const bool act = i < C.Rp;
    const TS *gz = static_cast<const TS *>(fp.spec) + C.spec + (size_t)f * R * C.Rp + i;
    const TS *sp = static_cast<const TS *>(fp.spec) + C.spec + (size_t)C.bins * R * C.Rp + (size_t)f * C.sp + i;
    constexpr int JW = kFftI / kFftW;
    const int jw0 = JW * w, jw1 = min(jw0 + JW, R);
    // double-buffered groups of SG rows with in-bounds loads in place of the
    // branches, as in k_fft_bins_sym (a lane past the padded rows has zero
    // weights, a lane past row j's stored part uses zeros)
    constexpr int SG = kFftSG;
    const int nfull = jw1 > jw0 ? (jw1 - jw0) / SG : 0;
    if (nfull > 0) {
        const TS *gzl = gz + (act ? 0 : C.Rp - 4 - i);
        Row4<TS> ga[SG], sa[SG], gb[SG], sb[SG];
        auto load = [&](Row4<TS>(&g)[SG], Row4<TS>(&sv)[SG], int j) {
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                const int jj = j + u, last = 4 * (jj >> 2);
                g[u].ld(gzl + (size_t)jj * C.Rp);
                sv[u].ld(sp - i + sym_row(jj) + min(i, last));
            }
        };
        auto comp = [&](const Row4<TS>(&g)[SG], const Row4<TS>(&sv)[SG], int j) {
            __builtin_amdgcn_sched_barrier(0);  // keep the loads above (see k_fft_bins)
            double re[SG], im[SG];
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                const int jj = j + u;
                const bool on = lane <= (jj >> 2);
                const double2 wj = sW[jj];
                re[u] = im[u] = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    re[u] = fma(g[u][t], wzr[t], re[u]);
                    im[u] = fma(g[u][t], wzi[t], im[u]);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double sv_t = on ? sv[u][t] : 0.0;
                    re[u] = fma(sv_t, wri[t], re[u]);
                    im[u] = fma(-sv_t, wrr[t], im[u]);
                    const double m = i + t < jj ? sv_t : 0.0;
                    ar[t] = fma(m, wj.y, ar[t]);
                    ai[t] = fma(-m, wj.x, ai[t]);
                }
            }
#pragma unroll
            for (int u = 0; u < SG; ++u) {
                re[u] = wave_sum(re[u]);
                im[u] = wave_sum(im[u]);
            }
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < SG; ++u) tD[j + u] = make_double2(re[u], im[u]);
            }
        };
        load(ga, sa, jw0);
        for (int k = 0; k + 1 < nfull; k += 2) {
            load(gb, sb, jw0 + SG * (k + 1));
            comp(ga, sa, jw0 + SG * k);
            load(ga, sa, jw0 + SG * min(k + 2, nfull - 1));
            comp(gb, sb, jw0 + SG * (k + 1));
        }
        if (nfull & 1) comp(ga, sa, jw0 + SG * (nfull - 1));
    }
    for (int j = jw0 + SG * nfull; j < jw1; j += 4) {
        double re[4], im[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            re[u] = im[u] = 0.0;
            const int jj = j + u;
            if (jj >= jw1) continue;  // uniform
            if (act) {
                double g[4];
                load4(gz + (size_t)jj * C.Rp, g);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    re[u] = fma(g[t], wzr[t], re[u]);
                    im[u] = fma(g[t], wzi[t], im[u]);
                }
            }
            if (lane <= (jj >> 2)) {
                const double2 wj = sW[jj];
                double sv[4];
                load4(sp + sym_row(jj), sv);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    re[u] = fma(sv[t], wri[t], re[u]);
                    im[u] = fma(-sv[t], wrr[t], im[u]);
                    const double m = i + t < jj ? sv[t] : 0.0;
                    ar[t] = fma(m, wj.y, ar[t]);
                    ai[t] = fma(-m, wj.x, ai[t]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            re[u] = wave_sum(re[u]);
            im[u] = wave_sum(im[u]);
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j + u < jw1) tD[j + u] = make_double2(re[u], im[u]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            red[w - 1][t][lane] = ar[t];
            red[w - 1][4 + t][lane] = ai[t];
        }
    }
    __syncthreads();
    if (w == 0) {
        double *out = fp.bpart + C.bpart + (size_t)f * 2;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (i + t < R) {
                double sr = ar[t], si = ai[t];
                for (int v = 0; v < kFftW - 1; ++v) {
                    sr += red[v][t][lane];
                    si += red[v][4 + t][lane];
                }
                out[(size_t)(i + t) * C.bins * 2] = tD[i + t].x + sr;
                out[(size_t)(i + t) * C.bins * 2 + 1] = tD[i + t].y + si;
            }
    }
}

// source rows a = 2q, b = 2q + 1: Y = out^_a + i out^_b (the target blocks
// summed in order), inverse DFT, partT[0][e] of both rows' elements
__global__ __launch_bounds__(256) void k_fft_rows_invT(FftPlan fp, const int *__restrict__ pub2int,
                                                       double *__restrict__ partT) {
    extern __shared__ double2 xs[];
    const int4 it = fp.items[blockIdx.x];
    const FftCoil C = fp.coils[it.x];
    const int a = 2 * it.y, b = a + 1;
    const bool hb = b < C.R;
    const double *bp = fp.bpart + C.bpart;
    inverse_pair(xs, C, fp, [&](int f, double &ur, double &ui, double &vr, double &vi) {
        ur = ui = vr = vi = 0.0;
        for (int ib = 0; ib < C.IB; ++ib) {
            const double *q = bp + (((size_t)ib * C.R + a) * C.bins + f) * 2;
            ur += q[0];
            ui += q[1];
            if (hb) {
                vr += q[C.bins * 2];
                vi += q[C.bins * 2 + 1];
            }
        }
    });
    const double invL = 1.0 / (double)C.L;
    const int *pa = pub2int + C.off + (size_t)a * C.Z;
    for (int z = threadIdx.x; z < C.Z; z += blockDim.x) {
        const double2 F = xs[z];
        partT[pa[z]] = F.x * invL;
        if (hb) partT[pa[C.Z + z]] = -F.y * invL;
    }
}

template <typename TS>
hipError_t field_fft(const DevState &s, const FftPlan &fp, const int *pub2int, hipStream_t st) {
    const size_t sh = (size_t)fp.Lmax * sizeof(double2);
    const int *none = nullptr;
    hipLaunchKernelGGL(k_fft_rows_fwd, dim3(fp.npairs), dim3(256), sh, st, fp, s.I, pub2int, 0, none);
    const int4 *bins = fp.items + fp.npairs + fp.nrows;
    if (fp.nbins) hipLaunchKernelGGL((k_fft_bins<TS, 0>), dim3(fp.nbins), dim3(64 * kFftW), 0, st, fp, bins, none);
    if (fp.nsym)
        hipLaunchKernelGGL(k_fft_bins_sym<TS>, dim3(fp.nsym), dim3(64 * kFftW), 0, st, fp, bins + fp.nbins + fp.nbinsT);
    hipLaunchKernelGGL(k_fft_rows_inv, dim3(fp.nrows), dim3(256), sh, st, fp, pub2int, s.part, 0, none);
    return hipGetLastError();
}

template <typename TS>
hipError_t fieldT_fft(const FftPlan &fp, const double *wr, const double *wz, const int *pub2int, double *partT,
                      hipStream_t st) {
    const size_t sh = (size_t)fp.Lmax * sizeof(double2);
    hipLaunchKernelGGL(k_fft_rows_fwdT, dim3(fp.nrows), dim3(256), sh, st, fp, wr, wz, pub2int);
    const int4 *binsT = fp.items + fp.npairs + fp.nrows + fp.nbins;
    if (fp.nbinsT) hipLaunchKernelGGL(k_fft_binsT<TS>, dim3(fp.nbinsT), dim3(256), 0, st, fp, binsT);
    if (fp.nsym) hipLaunchKernelGGL(k_fft_binsT_sym<TS>, dim3(fp.nsym), dim3(64 * kFftW), 0, st, fp, binsT + fp.nbinsT);
    hipLaunchKernelGGL(k_fft_rows_invT, dim3(fp.npairs), dim3(256), sh, st, fp, pub2int, partT);
    return hipGetLastError();
}

}  // namespace

void fft_plan(const std::vector<CoilDev> &coils, int flux, int prec, FftHostPlan &fp) {
    fp = FftHostPlan();
    fp.flux = flux;
    std::vector<int4> pairs, rows, bins, binsT, sym, all;
    auto up4 = [](size_t v) { return (v + 3) & ~size_t(3); };
    for (size_t ci = 0; ci < coils.size(); ++ci) {
        const CoilDev &d = coils[ci];
        FftCoil C{};
        C.R = d.layers * d.ne;
        C.Z = d.turns * d.ne;
        C.Rp = (C.R + 3) & ~3;
        int logL = 1;
        while ((1 << logL) < 2 * C.Z - 1) ++logL;
        C.L = 1 << logL;
        C.logL = logL;
        C.bins = C.L / 2 + 1;
        C.P = (C.R + kFftJ - 1) / kFftJ;
        C.IB = (C.Rp + kFftI - 1) / kFftI;
        C.off = d.off;
        C.kscale = d.kscale;
        C.kflux = kMu0 * d.d;
        C.c2d = d.c2d;
        // packed S where the pass is bound by the spectra's bytes: FP64 spectra
        // (C2 FP64 145 -> 132 us per pass); with FP32 spectra the wave sums
        // of the rows-above shares cost more than the bytes saved (67 -> 87 us)
        C.sym = prec == COIL_FP64 && C.Rp <= kFftI && C.R <= kFftJ ? 1 : 0;
        C.sp = sym_row(C.R);
        C.spec = fp.spec_reals;
        fp.spec_reals += up4((size_t)C.bins * C.R * C.Rp + (C.sym ? (size_t)C.bins * C.sp : (size_t)C.bins * C.R * C.Rp));
        C.fspec = fp.flux_reals;
        if (flux) fp.flux_reals += up4((size_t)C.bins * C.R * C.Rp);
        C.hat = fp.hat_reals;
        fp.hat_reals += up4((size_t)C.bins * C.Rp * 4);
        C.bpart = fp.bpart_reals;
        fp.bpart_reals += up4(std::max((size_t)C.P * C.bins * C.Rp * 4, (size_t)C.IB * C.bins * C.R * 2));
        fp.Lmax = std::max(fp.Lmax, C.L);
        const int nt = (C.Rp + kFftI - 1) / kFftI;
        for (int q = 0; q < (C.R + 1) / 2; ++q) pairs.push_back(make_int4((int)ci, q, 0, 0));
        for (int i = 0; i < C.R; ++i) rows.push_back(make_int4((int)ci, i, 0, 0));
        for (int f = 0; f < C.bins; ++f) {
            for (int tb = 0; tb < nt; ++tb)
                for (int p = 0; p < C.P; ++p) {
                    if (!C.sym) bins.push_back(make_int4((int)ci, f, tb, p));
                    all.push_back(make_int4((int)ci, f, tb, p));
                }
            if (C.sym) {
                sym.push_back(make_int4((int)ci, f, 0, 0));
                continue;
            }
            for (int jb = 0; jb < C.P; ++jb)
                for (int ib = 0; ib < C.IB; ++ib) binsT.push_back(make_int4((int)ci, f, jb, ib));
        }
        fp.coils.push_back(C);
    }
    fp.logLmax = 1;
    while ((1 << fp.logLmax) < fp.Lmax) ++fp.logLmax;
    fp.npairs = (int)pairs.size();
    fp.nrows = (int)rows.size();
    fp.nbins = (int)bins.size();
    fp.nbinsT = (int)binsT.size();
    fp.nsym = (int)sym.size();
    fp.nflux = (int)all.size();
    fp.items = pairs;
    for (const auto *v : {&rows, &bins, &binsT, &sym, &all}) fp.items.insert(fp.items.end(), v->begin(), v->end());
}

hipError_t launch_fft_setup(const DevState &s, const FftPlan &fp, const FftCoil *hc, int ncoils, void *tmp,
                            size_t tmp_bytes, hipStream_t st) {
    (void)s;
    double2 *t = static_cast<double2 *>(tmp);
    for (int c = 0; c < ncoils; ++c) {
        const FftCoil &C = hc[c];
        const size_t per_row = (size_t)C.R * C.bins * sizeof(double2);
        const int bs = (int)std::min<size_t>((size_t)C.R, tmp_bytes / per_row);
        if (bs < 1) return hipErrorInvalidValue;
        for (int kind = 0; kind < (fp.fspec ? 2 : 1); ++kind)
            for (int b0 = 0; b0 < C.R; b0 += bs) {
                const int nb = std::min(bs, C.R - b0);
                hipLaunchKernelGGL(k_fft_spec, dim3(C.R, nb), dim3(256), (size_t)C.L * sizeof(double2), st, fp, c,
                                   b0, t, kind);
                const dim3 g((C.bins + 31) / 32, (C.Rp + 31) / 32, nb);
                if (kind == 1)
                    hipLaunchKernelGGL(k_fft_spec_store<double>, g, dim3(256), 0, st, fp, c, b0, t,
                                       fp.fspec + C.fspec, 1);
                else if (fp.prec == COIL_MIXED)
                    hipLaunchKernelGGL(k_fft_spec_store<float>, g, dim3(256), 0, st, fp, c, b0, t,
                                       static_cast<float *>(fp.spec) + C.spec, 2);
                else
                    hipLaunchKernelGGL(k_fft_spec_store<double>, g, dim3(256), 0, st, fp, c, b0, t,
                                       static_cast<double *>(fp.spec) + C.spec, 2);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    }
    return hipSuccess;
}

hipError_t launch_field_fft(const DevState &s, const FftPlan &fp, const int *pub2int, hipStream_t st) {
    return fp.prec == COIL_MIXED ? field_fft<float>(s, fp, pub2int, st) : field_fft<double>(s, fp, pub2int, st);
}

hipError_t launch_flux_fft(const DevState &s, const FftPlan &fp, const double *v, const int *pub2int,
                           const int *done, hipStream_t st) {
    const size_t sh = (size_t)fp.Lmax * sizeof(double2);
    hipLaunchKernelGGL(k_fft_rows_fwd, dim3(fp.npairs), dim3(256), sh, st, fp, v, pub2int, 1, done);
    const int4 *all = fp.items + fp.npairs + fp.nrows + fp.nbins + fp.nbinsT + fp.nsym;
    hipLaunchKernelGGL((k_fft_bins<double, 1>), dim3(fp.nflux), dim3(64 * kFftW), 0, st, fp, all, done);
    hipLaunchKernelGGL(k_fft_rows_inv, dim3(fp.nrows), dim3(256), sh, st, fp, pub2int, s.part, 1, done);
    return hipGetLastError();
}

hipError_t launch_fieldT_fft(const DevState &s, const FftPlan &fp, const double *wr, const double *wz,
                             const int *pub2int, double *partT, hipStream_t st) {
    (void)s;
    return fp.prec == COIL_MIXED ? fieldT_fft<float>(fp, wr, wz, pub2int, partT, st)
                                 : fieldT_fft<double>(fp, wr, wz, pub2int, partT, st);
}

}  // namespace coilq
