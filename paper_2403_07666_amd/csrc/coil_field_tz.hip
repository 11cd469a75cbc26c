// coil_field_tz.hip -- field pass that evaluates each distinct Green's
// function value once per tile (z-translation invariance of the coaxial-ring
// kernel on a regular grid).
//
// For a coil on a regular (r, z) grid, the field of source (j_r, j_z) at
// target (i_r, i_z) depends only on (i_r, j_r, i_z - j_z): the ring Green's
// function is invariant under a common shift in z.  The all-pairs sum
//   B(i_r, i_z) = sum_{j_r, j_z} g(i_r, j_r, i_z - j_z) I(j_r, j_z)
// is therefore, for every pair of rows (i_r, j_r), a 1-D convolution along z.
// A work item owns one target row segment of 64*W consecutive z (one target
// per lane and W per thread) and an interleaved set of source rows; for every
// source row and every chunk of up to SMAX source z it
//   1. evaluates the 64*W + se distinct kernel values g(delta) on the fly
//      (elliptic integrals as in the direct pass; mixed precision: FP32 where
//      m1 >= m1_near, the near values FP64 from a table made once at set-up)
//      into LDS, stored de-interleaved by delta mod W so that every lane reads
//      a different bank, and copies the entries whose mirror -delta is
//      already there (g_r odd, g_z even);
//   2. streams the source currents through LDS and accumulates
//      acc[c] += g(delta) * I with a W-register sliding window over delta:
//      one LDS read of g feeds 2W FMAs.
// Every pair still contributes g * I exactly once; only redundant evaluations
// of identical kernel values are removed.  FP64 mode keeps the table, the
// currents and the accumulation in FP64.  Mixed mode stores the kernel values
// (FP32 far, FP64 near, both rounded to FP32) and the currents in FP32 and
// runs the pair products and partial sums in FP32 (non-packed FP32 FMA issues
// at twice the FP64 rate on this GPU), adding the partial sums of every 16W
// sources into FP64 accumulators.
#include <hip/hip_runtime.h>

#include <climits>

#include "coil_device.h"
#include "coil_field_tz.h"

namespace coilq {

// a x + c with the constant c as a scalar-register operand.  Left to itself
// the compiler keeps the 44 FP64 coefficients in vector registers for the
// whole kernel and copies one before every v_fmac_f64 of a Horner step.
__device__ __forceinline__ double fma_sc(double a, double x, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(x), "s"(c));
    return r;
}

template <int N>
__device__ __forceinline__ double horner_sc(const double (&c)[N], double x) {
    double a = fma_sc(x, c[0], c[1]);
#pragma unroll
    for (int k = 2; k < N; ++k) a = fma_sc(a, x, c[k]);
    return a;
}

// unit-current kernel values (grid units): f g_r, f g_z as in pair64/pair32
__device__ __forceinline__ double2 kern64(double dr, double dz, double sr) {
    const double dz2 = dz * dz;
    const double al2 = fma(dr, dr, dz2);
    const double be2 = fma(sr, sr, dz2);
    if (!(al2 > 0.0)) return make_double2(0.0, 0.0);  // the element's own ring
    const double rb = rsqrt(be2);
    const double m1 = al2 * (rb * rb);
    const double L = -log(m1);
    const double K = fma(horner_sc(ellipk64_Q_c, m1), L, horner_sc(ellipk64_P_c, m1));
    const double E = fma(horner_sc(ellipe64_Q_c, m1), L, horner_sc(ellipe64_P_c, m1));
    const double f = rb / al2;
    const double alK = al2 * K;
    const double gz = fma(fma(-dr, sr, -dz2), E, alK);
    const double gr = dz * fma(0.5 * (al2 + be2), E, -alK);
    return make_double2(f * gr, f * gz);
}

// Flux kernel (unit source strength mu0 d): the mutual inductance of two
// coaxial rings, Maxwell's M = mu0 be [ (1 + m1)/2 K - E ] with be in grid
// units times d, as (0, M / (mu0 d)); even in dz.  The element's own ring
// (al2 = 0) is left out (its self inductance is added by the caller).
__device__ __forceinline__ double2 kernflux64(double dr, double dz, double sr) {
    const double dz2 = dz * dz;
    const double al2 = fma(dr, dr, dz2);
    const double be2 = fma(sr, sr, dz2);
    if (!(al2 > 0.0)) return make_double2(0.0, 0.0);
    const double rb = rsqrt(be2);
    const double m1 = al2 * (rb * rb);
    const double L = -log(m1);
    const double K = fma(horner_sc(ellipk64_Q_c, m1), L, horner_sc(ellipk64_P_c, m1));
    const double E = fma(horner_sc(ellipe64_Q_c, m1), L, horner_sc(ellipe64_P_c, m1));
    return make_double2(0.0, sqrt(be2) * fma(0.5 * (1.0 + m1), K, -E));
}

__device__ __forceinline__ float2 kern32(float dr, float dz, float sr) {
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
    return make_float2(f * gr, f * gz);
}

// Table of kernel values g(delta) for delta = dlo + tau, tau in [0, nt),
// stored at [(tau % W) * Q + tau / W].  g_z is even and g_r odd in delta
// (g_z depends on delta^2 only, g_r on delta times the same factor, and the
// near/far choice on delta^2), so an entry whose mirror -delta lies in the
// table is copied from it with g_r negated: bitwise the value a direct
// evaluation gives.  When the table spans a whole row pair (targets and
// sources of one z segment) about half of the entries are copies.
__device__ __forceinline__ void put(double2 *p, double2 v) { *p = v; }
__device__ __forceinline__ void put(float2 *p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ void put(double2 *p, float2 v) { *p = make_double2(v.x, v.y); }
__device__ __forceinline__ void put(float2 *p, float2 v) { *p = v; }

// Mixed precision: g is evaluated in FP32 except near k -> 1, where it is
// taken from the pair's table of FP64 values made at set-up (np = (first
// entry, count) for this pair of rows; |delta| < count is near).  The values
// there are those a direct FP64 evaluation gives, rounded to FP32, and g_r is
// odd in delta, so the entry for -delta is the stored one with g_r negated.
template <int MIXED, int W, int Q, bool NEG = false, int KIND = 0, typename T2>
__device__ __forceinline__ void fill_table(T2 *gt, int lane, int nt, int dlo, double dr, double sr, int2 np,
                                           const float2 *__restrict__ nv) {
    const float drf = (float)dr, srf = (float)sr;
    for (int tau = lane; tau < nt; tau += 64) {
        const int delta = dlo + tau;
        const int mt = -delta - dlo;  // table index of -delta
        if (delta >= 0 || mt >= nt) {
            const int dz = NEG ? -delta : delta;
            T2 *p = &gt[(tau % W) * Q + tau / W];
            if (KIND == 1) {
                put(p, kernflux64(dr, (double)dz, sr));
            } else if (!MIXED) {
                put(p, kern64(dr, (double)dz, sr));
            } else {
                const int a = dz < 0 ? -dz : dz;
                if (a < np.y) {
                    float2 v = nv[np.x + a];
                    if (dz < 0) v.x = -v.x;
                    put(p, v);
                } else {
                    put(p, kern32(drf, (float)dz, srf));
                }
            }
        }
    }
    __syncthreads();
    for (int tau = lane; tau < nt; tau += 64) {
        const int delta = dlo + tau;
        const int mt = -delta - dlo;
        if (delta < 0 && mt < nt) {
            T2 v = gt[(mt % W) * Q + mt / W];
            v.x = -v.x;
            gt[(tau % W) * Q + tau / W] = v;
        }
    }
}

// Forward pass shape: 64 W targets per item; sources in chunks of up to SMAX
// (a whole row of the benchmark coils, so that the mirror halves the table);
// the table holds TZ + se entries for a chunk of se sources (se = the chunk
// length rounded up to W), W * Q of them at most.  For W = 8 table and
// currents take 20 KiB in FP64 (eight items in the 160 KiB of LDS of a CU)
// and 10 KiB in mixed precision (sixteen).
template <int W>
struct TzShape {
    static constexpr int SMAX = W >= 5 ? 512 : 256;
    static constexpr int SMAXW = (SMAX + W - 1) / W * W;  // a chunk rounded up to W
    static constexpr int TZ = 64 * W;
    static constexpr int Q = (TZ + SMAXW) / W;
};

// One block of W sources t = W tb + u.  Target cc of a lane reads entry
// tau = W (lane - tb + se / W) + cc - u, whose residue (cc - u) mod W names its
// ring register; after source u the entry leaving the window (residue
// W - 1 - u) is replaced by the one entering it, whose quotient is
// base = lane - tb + se / W - 1 for every u of the block.
template <int W, int Q>
__device__ __forceinline__ void tz_block(const double2 *gt, double2 (&ring)[W], double (&ar)[W],
                                         double (&az)[W], const double (&Iv)[W], int base) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
        const double I = Iv[u];
#pragma unroll
        for (int cc = 0; cc < W; ++cc) {
            const double2 g = ring[(cc - u + W) % W];
            ar[cc] = fma(g.x, I, ar[cc]);
            az[cc] = fma(g.y, I, az[cc]);
        }
        ring[(W - 1 - u) % W] = gt[((W - 1 - u) % W) * Q + base];
    }
}

// One forward item of width W; gt and Is point into the launch's LDS buffer.
// Wave priority by progress through the item.  The SIMD's arbiter issues the
// oldest ready wave first, so of the waves sharing a SIMD the oldest would
// finish first and the youngest would run last, alone, at a fraction of the
// SIMD's FP32 rate.  Lowering a wave's priority as it works through its rows
// keeps the waves of a SIMD level, so they finish together (measured: 2-4 %
// off the forward pass).  The arithmetic is unchanged.
__device__ __forceinline__ void prio_by_progress(int done, int total) {
    const int lv = (4 * done) / total;
    if (lv <= 0)
        __builtin_amdgcn_s_setprio(3);
    else if (lv == 1)
        __builtin_amdgcn_s_setprio(2);
    else if (lv == 2)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

template <int MIXED, int W, int KIND = 0>
__device__ __forceinline__ void tz_item(const DevState &s, const RunConst &rc, const TzItem &item,
                                        const int *__restrict__ rows, const double *__restrict__ Ipub,
                                        const int *__restrict__ pub2int, double2 *gt, double *Is) {
    using Sh = TzShape<W>;
    constexpr int SMAX = Sh::SMAX, TZ = Sh::TZ, Q = Sh::Q;
    const int lane = threadIdx.x;
    {
        const CoilDev c = s.coils[item.coil];
        const int nz = c.turns * c.ne;
        const int ir = item.ir, z0 = item.z0;
        double ar[W], az[W];
#pragma unroll
        for (int cc = 0; cc < W; ++cc) ar[cc] = az[cc] = 0.0;
        // the item's source rows: a run of the coil's rows in bit-reversed order,
        // so that every item of a target row gets a like share of the near rows
        for (int k = 0; k < item.rcnt; ++k) {
            prio_by_progress(k, item.rcnt);
            const int jr = rows[item.roff + k];
            const double dr = (double)(ir - jr);
            const double sr = c.c2d + (double)(ir + jr);
            const int2 np = MIXED ? s.near_pair[c.near_base + ir * (c.layers * c.ne) + jr] : make_int2(0, 0);
            const double *Irow = Ipub + c.off + (size_t)jr * nz;
            for (int s0 = 0; s0 < nz; s0 += SMAX) {
                const int sn = min(SMAX, nz - s0);
                const int nb = (sn + W - 1) / W;
                const int se = nb * W;
                // delta = z_target - z_source = dlo + tau
                const int dlo = z0 - s0 - se;
                __syncthreads();
                fill_table<MIXED, W, Q, false, KIND>(gt, lane, TZ + se, dlo, dr, sr, np, s.near_val);
                const double scale = KIND == 1 ? kMu0 * c.d : c.kscale;
                for (int t = lane; t < se; t += 64) Is[t] = t < sn ? scale * Irow[s0 + t] : 0.0;
                __syncthreads();
                double2 ring[W];
#pragma unroll
                for (int cc = 0; cc < W; ++cc) ring[cc] = gt[cc * Q + lane + nb];
                // the W currents of block tb + 1 are read while block tb is
                // accumulated (two register sets, the loop unrolled twice)
                double Ia[W], Ib[W];
#pragma unroll
                for (int u = 0; u < W; ++u) Ia[u] = Is[u];
                for (int tb = 0; tb < nb; tb += 2) {
                    if (tb + 1 < nb) {
#pragma unroll
                        for (int u = 0; u < W; ++u) Ib[u] = Is[(tb + 1) * W + u];
                    }
                    tz_block<W, Q>(gt, ring, ar, az, Ia, lane - tb + nb - 1);
                    if (tb + 1 < nb) {
                        if (tb + 2 < nb) {
#pragma unroll
                            for (int u = 0; u < W; ++u) Ia[u] = Is[(tb + 2) * W + u];
                        }
                        tz_block<W, Q>(gt, ring, ar, az, Ib, lane - tb + nb - 2);
                    }
                }
            }
        }
#pragma unroll
        for (int cc = 0; cc < W; ++cc) {
            const int z = z0 + W * lane + cc;
            if (z < nz) {
                const int e = pub2int[c.off + ir * nz + z];
                s.part[(size_t)item.slot * s.N + e] = make_double2(ar[cc], az[cc]);
            }
        }
    }
}

template <int W, int Q>
__device__ __forceinline__ void tz_block32(const float2 *gt, float2 (&ring)[W], float (&br)[W], float (&bz)[W],
                                           const float (&Iv)[W], int base) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
        const float I = Iv[u];
#pragma unroll
        for (int cc = 0; cc < W; ++cc) {
            const float2 g = ring[(cc - u + W) % W];
            br[cc] = fmaf(g.x, I, br[cc]);
            bz[cc] = fmaf(g.y, I, bz[cc]);
        }
        ring[(W - 1 - u) % W] = gt[((W - 1 - u) % W) * Q + base];
    }
}

// Mixed precision: the kernel values (FP32 far, FP64 near, both rounded to
// FP32), the currents and the products are FP32; every 16W sources the FP32
// partial sums are added into FP64 accumulators.
template <int W>
__device__ __forceinline__ void tz_item32(const DevState &s, const RunConst &rc, const TzItem &item,
                                          const int *__restrict__ rows, const float *__restrict__ Ipub32,
                                          const int *__restrict__ pub2int, float2 *gt, float *Is) {
    using Sh = TzShape<W>;
    constexpr int SMAX = Sh::SMAX, TZ = Sh::TZ, Q = Sh::Q;
    const int lane = threadIdx.x;
    const CoilDev c = s.coils[item.coil];
    const int nz = c.turns * c.ne;
    const int ir = item.ir, z0 = item.z0;
    double ar[W], az[W];
#pragma unroll
    for (int cc = 0; cc < W; ++cc) ar[cc] = az[cc] = 0.0;
    for (int k = 0; k < item.rcnt; ++k) {
        prio_by_progress(k, item.rcnt);
        const int jr = rows[item.roff + k];
        const double dr = (double)(ir - jr);
        const double sr = c.c2d + (double)(ir + jr);
        const int2 np = s.near_pair[c.near_base + ir * (c.layers * c.ne) + jr];
        const float *Irow = Ipub32 + c.off + (size_t)jr * nz;
        for (int s0 = 0; s0 < nz; s0 += SMAX) {
            const int sn = min(SMAX, nz - s0);
            const int nb = (sn + W - 1) / W;
            const int se = nb * W;
            const int dlo = z0 - s0 - se;
            __syncthreads();
            fill_table<1, W, Q>(gt, lane, TZ + se, dlo, dr, sr, np, s.near_val);
            for (int t = lane; t < se; t += 64) Is[t] = t < sn ? Irow[s0 + t] : 0.0f;
            __syncthreads();
            float2 ring[W];
#pragma unroll
            for (int cc = 0; cc < W; ++cc) ring[cc] = gt[cc * Q + lane + nb];
            float Ia[W], Ib[W], br[W], bz[W];
#pragma unroll
            for (int u = 0; u < W; ++u) Ia[u] = Is[u];
#pragma unroll
            for (int cc = 0; cc < W; ++cc) br[cc] = bz[cc] = 0.0f;
            for (int tb = 0; tb < nb; tb += 2) {
                if (tb + 1 < nb) {
#pragma unroll
                    for (int u = 0; u < W; ++u) Ib[u] = Is[(tb + 1) * W + u];
                }
                tz_block32<W, Q>(gt, ring, br, bz, Ia, lane - tb + nb - 1);
                if (tb + 1 < nb) {
                    if (tb + 2 < nb) {
#pragma unroll
                        for (int u = 0; u < W; ++u) Ia[u] = Is[(tb + 2) * W + u];
                    }
                    tz_block32<W, Q>(gt, ring, br, bz, Ib, lane - tb + nb - 2);
                }
                if ((tb & 14) == 14 || tb + 2 >= nb) {  // after every 16 blocks, and at the end
#pragma unroll
                    for (int cc = 0; cc < W; ++cc) {
                        ar[cc] += (double)br[cc];
                        az[cc] += (double)bz[cc];
                        br[cc] = bz[cc] = 0.0f;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < W; ++cc) {
        const int z = z0 + W * lane + cc;
        if (z < nz) s.part[(size_t)item.slot * s.N + pub2int[c.off + ir * nz + z]] = make_double2(ar[cc], az[cc]);
    }
}

// LDS of one item: the widest table plus its chunk of currents (W = 8: 20 KiB,
// so eight items share the 160 KiB of a CU)
constexpr int kTzLds2 = 20480 / 16;
template <int W>
constexpr bool tz_fits() {
    return TzShape<W>::Q * W * 16 + TzShape<W>::SMAXW * 8 <= kTzLds2 * 16;
}

// All widths in one launch: items are ordered widest first, and each
// workgroup branches (uniformly) on its item's width.
// Work items of a workgroup.  Workgroup b starts with item b.  With a ticket
// counter (the default launch, one workgroup per slot of the GPU) it then
// takes the next item in list order whenever it is free, so the parts of the
// GPU that run faster take more of them (the counter starts at 0 and hands out
// items from gridDim.x on); without one it strides by the grid.  Items write
// disjoint outputs, so the results do not depend on which workgroup takes
// which item.
__device__ __forceinline__ int next_item(int *ticket, int it) {
    if (!ticket) return it + (int)gridDim.x;
    int t = 0;
    if (threadIdx.x == 0) t = atomicAdd(ticket, 1);
    return (int)gridDim.x + __builtin_amdgcn_readfirstlane(t);
}
__device__ __forceinline__ int first_item(int *) { return (int)blockIdx.x; }

template <int MIXED, int KIND = 0>
__device__ __forceinline__ void field_tz_items(const DevState &s, const RunConst &rc,
                                               const TzItem *__restrict__ items, const int *__restrict__ rows,
                                               int nitems, const double *__restrict__ Ipub,
                                               const float *__restrict__ Ipub32,
                                               const int *__restrict__ pub2int, double2 *lds, int *ticket) {
    for (int it = first_item(ticket); it < nitems; it = next_item(ticket, it)) {
        const TzItem item = items[it];
#define COILQ_TZ_CASE(Wv)                                                                                   \
    case Wv:                                                                                                \
        static_assert(tz_fits<Wv>(), "LDS");                                                                \
        if (MIXED)                                                                                          \
            tz_item32<Wv>(s, rc, item, rows, Ipub32, pub2int, reinterpret_cast<float2 *>(lds),              \
                          reinterpret_cast<float *>(reinterpret_cast<float2 *>(lds) + TzShape<Wv>::Q * Wv)); \
        else                                                                                                \
            tz_item<MIXED, Wv, KIND>(s, rc, item, rows, Ipub, pub2int, lds,                                 \
                               reinterpret_cast<double *>(lds + TzShape<Wv>::Q * Wv));                      \
        break;
        switch (item.w) {
            COILQ_TZ_CASE(8)
            COILQ_TZ_CASE(7)
            COILQ_TZ_CASE(6)
            COILQ_TZ_CASE(5)
            COILQ_TZ_CASE(4)
            COILQ_TZ_CASE(3)
            COILQ_TZ_CASE(2)
        }
#undef COILQ_TZ_CASE
    }
}

// Mixed precision: 10 KiB of LDS per item and at most 128 VGPRs, so four
// waves per SIMD; the register limit spills a few addresses, reloaded per
// row, none in the FMA loop.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_field_tz32(
    DevState s, RunConst rc, const TzItem *__restrict__ items, const int *__restrict__ rows, int nitems,
    const float *__restrict__ Ipub32, const int *__restrict__ pub2int, int *ticket) {
    __shared__ double2 lds[kTzLds2 / 2];
    field_tz_items<1>(s, rc, items, rows, nitems, nullptr, Ipub32, pub2int, lds, ticket);
}

__global__ __launch_bounds__(64) void k_field_tz64(DevState s, RunConst rc, const TzItem *__restrict__ items,
                                                   const int *__restrict__ rows, int nitems,
                                                   const double *__restrict__ Ipub,
                                                   const int *__restrict__ pub2int, int *ticket) {
    __shared__ double2 lds[kTzLds2];
    field_tz_items<0>(s, rc, items, rows, nitems, Ipub, nullptr, pub2int, lds, ticket);
}

// Flux pass of the fully coupled A-V solve: part[slot][e].y = sum over the
// item's source rows of M(e, j) v_j / (mu0 d) * mu0 d, i.e. the off-diagonal
// inductance matrix times the vector v (public order in vpub), FP64.  Returns
// at once when the solve has converged (*done != 0).
__global__ __launch_bounds__(64) void k_flux_tz64(DevState s, RunConst rc, const TzItem *__restrict__ items,
                                                  const int *__restrict__ rows, int nitems,
                                                  const double *__restrict__ vpub, const int *__restrict__ pub2int,
                                                  int *ticket, const int *__restrict__ done) {
    if (*done) return;
    __shared__ double2 lds[kTzLds2];
    field_tz_items<0, 1>(s, rc, items, rows, nitems, vpub, nullptr, pub2int, lds, ticket);
}

// Transposed pass (adjoint): out(j_r, j_z) = sum over target rows i_r and
// targets i_z of g_r(i_r, j_r, i_z - j_z) wr(i_r, i_z) + g_z(...) wz(i_r, i_z).
// With d = j_z - i_z this is, for every pair of rows, the same convolution as
// the forward pass with the kernel G(d) = g(i_r, j_r, -d) (G_r odd, G_z even,
// so the mirror fill applies) and two weights per source.  Item fields: ir =
// output row j_r, z0 = output segment, summed rows rows[roff .. roff + rcnt).
// Chunks of up to 384 summed targets keep table and weights within 20 KiB
// (eight items per CU).
template <int W>
struct TzShapeT {
    static constexpr int SMAX = 384;
    static constexpr int SMAXW = (SMAX + W - 1) / W * W;
    static constexpr int TZ = 64 * W;
    static constexpr int Q = (TZ + SMAXW) / W;
};

template <int W, int Q>
__device__ __forceinline__ void tzT_block(const double2 *gt, double2 (&ring)[W], double (&acc)[W],
                                          const double2 (&wv)[W], int base) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
#pragma unroll
        for (int cc = 0; cc < W; ++cc) {
            const double2 g = ring[(cc - u + W) % W];
            acc[cc] = fma(g.x, wv[u].x, fma(g.y, wv[u].y, acc[cc]));
        }
        ring[(W - 1 - u) % W] = gt[((W - 1 - u) % W) * Q + base];
    }
}

template <int MIXED, int W>
__device__ __forceinline__ void tzT_item(const DevState &s, const RunConst &rc, const TzItem &item,
                                         const int *__restrict__ rows,
                                         const double *__restrict__ wr_pub, const double *__restrict__ wz_pub,
                                         const int *__restrict__ pub2int, double *partT, double2 *gt,
                                         double2 *ws) {
    using Sh = TzShapeT<W>;
    constexpr int SMAX = Sh::SMAX, TZ = Sh::TZ, Q = Sh::Q;
    const int lane = threadIdx.x;
    {
        const CoilDev c = s.coils[item.coil];
        const int nz = c.turns * c.ne;
        const int jr = item.ir, z0 = item.z0;
        double acc[W];
#pragma unroll
        for (int cc = 0; cc < W; ++cc) acc[cc] = 0.0;
        for (int k = 0; k < item.rcnt; ++k) {
            prio_by_progress(k, item.rcnt);
            const int ir = rows[item.roff + k];
            const double dr = (double)(ir - jr);
            const double sr = c.c2d + (double)(ir + jr);
            const int2 np = MIXED ? s.near_pair[c.near_base + ir * (c.layers * c.ne) + jr] : make_int2(0, 0);
            const size_t rowoff = c.off + (size_t)ir * nz;
            for (int s0 = 0; s0 < nz; s0 += SMAX) {
                const int sn = min(SMAX, nz - s0);
                const int nb = (sn + W - 1) / W;
                const int se = nb * W;
                // d = j_z - i_z = dlo + tau; entries hold g(i_r, j_r, -d)
                const int dlo = z0 - s0 - se;
                __syncthreads();
                fill_table<MIXED, W, Q, true>(gt, lane, TZ + se, dlo, dr, sr, np, s.near_val);
                for (int t = lane; t < se; t += 64)
                    ws[t] = t < sn ? make_double2(wr_pub[rowoff + s0 + t], wz_pub[rowoff + s0 + t])
                                   : make_double2(0.0, 0.0);
                __syncthreads();
                double2 ring[W];
#pragma unroll
                for (int cc = 0; cc < W; ++cc) ring[cc] = gt[cc * Q + lane + nb];
                double2 wa[W], wb[W];
#pragma unroll
                for (int u = 0; u < W; ++u) wa[u] = ws[u];
                for (int tb = 0; tb < nb; tb += 2) {
                    if (tb + 1 < nb) {
#pragma unroll
                        for (int u = 0; u < W; ++u) wb[u] = ws[(tb + 1) * W + u];
                    }
                    tzT_block<W, Q>(gt, ring, acc, wa, lane - tb + nb - 1);
                    if (tb + 1 < nb) {
                        if (tb + 2 < nb) {
#pragma unroll
                            for (int u = 0; u < W; ++u) wa[u] = ws[(tb + 2) * W + u];
                        }
                        tzT_block<W, Q>(gt, ring, acc, wb, lane - tb + nb - 2);
                    }
                }
            }
        }
#pragma unroll
        for (int cc = 0; cc < W; ++cc) {
            const int z = z0 + W * lane + cc;
            if (z < nz) partT[(size_t)item.slot * s.N + pub2int[c.off + jr * nz + z]] = acc[cc];
        }
    }
}

template <int W, int Q>
__device__ __forceinline__ void tzT_block32(const float2 *gt, float2 (&ring)[W], float (&bacc)[W],
                                            const float2 (&wv)[W], int base) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
#pragma unroll
        for (int cc = 0; cc < W; ++cc) {
            const float2 g = ring[(cc - u + W) % W];
            bacc[cc] = fmaf(g.x, wv[u].x, fmaf(g.y, wv[u].y, bacc[cc]));
        }
        ring[(W - 1 - u) % W] = gt[((W - 1 - u) % W) * Q + base];
    }
}

// Mixed precision transposed item: FP32 table, weights, products and partial
// sums, the partial sums of every 16W sources added into FP64 accumulators.
template <int W>
__device__ __forceinline__ void tzT_item32(const DevState &s, const RunConst &rc, const TzItem &item,
                                           const int *__restrict__ rows, const double *__restrict__ wr_pub,
                                           const double *__restrict__ wz_pub, const int *__restrict__ pub2int,
                                           double *partT, float2 *gt, float2 *ws) {
    using Sh = TzShapeT<W>;
    constexpr int SMAX = Sh::SMAX, TZ = Sh::TZ, Q = Sh::Q;
    const int lane = threadIdx.x;
    const CoilDev c = s.coils[item.coil];
    const int nz = c.turns * c.ne;
    const int jr = item.ir, z0 = item.z0;
    double acc[W];
#pragma unroll
    for (int cc = 0; cc < W; ++cc) acc[cc] = 0.0;
    for (int k = 0; k < item.rcnt; ++k) {
        prio_by_progress(k, item.rcnt);
        const int ir = rows[item.roff + k];
        const double dr = (double)(ir - jr);
        const double sr = c.c2d + (double)(ir + jr);
        const int2 np = s.near_pair[c.near_base + ir * (c.layers * c.ne) + jr];
        const size_t rowoff = c.off + (size_t)ir * nz;
        for (int s0 = 0; s0 < nz; s0 += SMAX) {
            const int sn = min(SMAX, nz - s0);
            const int nb = (sn + W - 1) / W;
            const int se = nb * W;
            const int dlo = z0 - s0 - se;
            __syncthreads();
            fill_table<1, W, Q, true>(gt, lane, TZ + se, dlo, dr, sr, np, s.near_val);
            for (int t = lane; t < se; t += 64)
                ws[t] = t < sn ? make_float2((float)wr_pub[rowoff + s0 + t], (float)wz_pub[rowoff + s0 + t])
                               : make_float2(0.0f, 0.0f);
            __syncthreads();
            float2 ring[W];
#pragma unroll
            for (int cc = 0; cc < W; ++cc) ring[cc] = gt[cc * Q + lane + nb];
            float2 wa[W], wb[W];
            float bacc[W];
#pragma unroll
            for (int u = 0; u < W; ++u) wa[u] = ws[u];
#pragma unroll
            for (int cc = 0; cc < W; ++cc) bacc[cc] = 0.0f;
            for (int tb = 0; tb < nb; tb += 2) {
                if (tb + 1 < nb) {
#pragma unroll
                    for (int u = 0; u < W; ++u) wb[u] = ws[(tb + 1) * W + u];
                }
                tzT_block32<W, Q>(gt, ring, bacc, wa, lane - tb + nb - 1);
                if (tb + 1 < nb) {
                    if (tb + 2 < nb) {
#pragma unroll
                        for (int u = 0; u < W; ++u) wa[u] = ws[(tb + 2) * W + u];
                    }
                    tzT_block32<W, Q>(gt, ring, bacc, wb, lane - tb + nb - 2);
                }
                if ((tb & 14) == 14 || tb + 2 >= nb) {  // after every 16 blocks, and at the end
#pragma unroll
                    for (int cc = 0; cc < W; ++cc) {
                        acc[cc] += (double)bacc[cc];
                        bacc[cc] = 0.0f;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < W; ++cc) {
        const int z = z0 + W * lane + cc;
        if (z < nz) partT[(size_t)item.slot * s.N + pub2int[c.off + jr * nz + z]] = acc[cc];
    }
}

constexpr int kTzTLds2 = 20480 / 16;
template <int W>
constexpr bool tzT_fits() {
    return TzShapeT<W>::Q * W * 16 + TzShapeT<W>::SMAXW * 16 <= kTzTLds2 * 16;
}

template <int MIXED>
__device__ __forceinline__ void fieldT_tz_items(const DevState &s, const RunConst &rc,
                                                const TzItem *__restrict__ items, const int *__restrict__ rows,
                                                int nitems, const double *__restrict__ wr_pub,
                                                const double *__restrict__ wz_pub,
                                                const int *__restrict__ pub2int, double *partT, double2 *lds,
                                                int *ticket) {
    for (int it = first_item(ticket); it < nitems; it = next_item(ticket, it)) {
        const TzItem item = items[it];
#define COILQ_TZT_CASE(Wv)                                                                                  \
    case Wv:                                                                                                \
        static_assert(tzT_fits<Wv>(), "LDS");                                                               \
        if (MIXED)                                                                                          \
            tzT_item32<Wv>(s, rc, item, rows, wr_pub, wz_pub, pub2int, partT,                              \
                           reinterpret_cast<float2 *>(lds),                                                 \
                           reinterpret_cast<float2 *>(lds) + TzShapeT<Wv>::Q * Wv);                         \
        else                                                                                                \
            tzT_item<MIXED, Wv>(s, rc, item, rows, wr_pub, wz_pub, pub2int, partT, lds,                    \
                                lds + TzShapeT<Wv>::Q * Wv);                                                \
        break;
        switch (item.w) {
            COILQ_TZT_CASE(8)
            COILQ_TZT_CASE(7)
            COILQ_TZT_CASE(6)
            COILQ_TZT_CASE(5)
            COILQ_TZT_CASE(4)
            COILQ_TZT_CASE(3)
            COILQ_TZT_CASE(2)
        }
#undef COILQ_TZT_CASE
    }
}

// as the forward mixed kernel: 10 KiB of LDS and at most 128 VGPRs per item
// (four waves per SIMD, spills outside the FMA loop)
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_fieldT_tz32(
    DevState s, RunConst rc, const TzItem *__restrict__ items, const int *__restrict__ rows, int nitems,
    const double *__restrict__ wr_pub, const double *__restrict__ wz_pub, const int *__restrict__ pub2int,
    double *partT, int *ticket) {
    __shared__ double2 lds[kTzTLds2 / 2];
    fieldT_tz_items<1>(s, rc, items, rows, nitems, wr_pub, wz_pub, pub2int, partT, lds, ticket);
}

__global__ __launch_bounds__(64) void k_fieldT_tz64(DevState s, RunConst rc, const TzItem *__restrict__ items,
                                                    const int *__restrict__ rows, int nitems,
                                                    const double *__restrict__ wr_pub,
                                                    const double *__restrict__ wz_pub,
                                                    const int *__restrict__ pub2int, double *partT,
                                                    int *ticket) {
    __shared__ double2 lds[kTzTLds2];
    fieldT_tz_items<0>(s, rc, items, rows, nitems, wr_pub, wz_pub, pub2int, partT, lds, ticket);
}

// I in public (row-major) order for the convolution pass, and (if Ipub32)
// kscale * I of the element's coil rounded to FP32 for the mixed pass; also
// clears the pass's ticket counter (if any) before the pass starts
__global__ void k_to_pub(const double *I, const int *perm, int n, double *Ipub, int *ticket, float *Ipub32,
                         const int *elem_coil, const CoilDev *coils) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double v = I[i];
        const int pub = perm[i];
        Ipub[pub] = v;
        if (Ipub32) Ipub32[pub] = (float)(coils[elem_coil[i]].kscale * v);
    }
    if (ticket && i == 0) *ticket = 0;
}

// Near kernel values of one coil: one workgroup per pair (a, b) of its rows,
// g(a - b, delta) for delta = 0 .. count - 1 in FP64, rounded to FP32.
__global__ __launch_bounds__(64) void k_near_fill(DevState s, int coil, int nr) {
    const CoilDev c = s.coils[coil];
    const int pr = blockIdx.x;
    const int a = pr / nr, b = pr - a * nr;
    const int2 np = s.near_pair[c.near_base + pr];
    const double dr = (double)(a - b), sr = c.c2d + (double)(a + b);
    float2 *out = const_cast<float2 *>(s.near_val) + np.x;
    for (int d = threadIdx.x; d < np.y; d += 64) {
        const double2 v = kern64(dr, (double)d, sr);
        out[d] = make_float2((float)v.x, (float)v.y);
    }
}

hipError_t launch_near_fill(const DevState &s, int coil, int nr, hipStream_t st) {
    if (nr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_near_fill, dim3(nr * nr), dim3(64), 0, st, s, coil, nr);
    return hipGetLastError();
}

hipError_t tz_resident_grids(TzPlan &tp) {
    int dev = 0, cus = 0, b = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_field_tz32, 64, 0)) != hipSuccess) return e;
    tp.grid32 = b * cus;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_field_tz64, 64, 0)) != hipSuccess) return e;
    tp.grid64 = b * cus;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_fieldT_tz32, 64, 0)) != hipSuccess) return e;
    tp.gridT32 = b * cus;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_fieldT_tz64, 64, 0)) != hipSuccess) return e;
    tp.gridT64 = b * cus;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_flux_tz64, 64, 0)) != hipSuccess) return e;
    tp.gridF64 = b * cus;
    return hipSuccess;
}

// one workgroup per resident slot with the ticket counter, or per item without
static int queue_grid(int slots, int n) { return slots > 0 ? min(slots, n) : n; }

hipError_t launch_field_tz_prep(const DevState &s, const TzPlan &tp, double *Ipub, hipStream_t st) {
    hipLaunchKernelGGL(k_to_pub, dim3((s.N + 255) / 256), dim3(256), 0, st, s.I, s.perm, s.N, Ipub, tp.ticket,
                       tp.Ipub32, s.elem_coil, s.coils);
    return hipGetLastError();
}

hipError_t launch_field_tz(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *Ipub,
                           const int *pub2int, int grid_limit, hipStream_t st) {
    hipError_t e = launch_field_tz_prep(s, tp, const_cast<double *>(Ipub), st);
    if (e != hipSuccess) return e;
    return launch_field_tz_kernel(s, rc, tp, Ipub, pub2int, grid_limit, st);
}

hipError_t launch_field_tz_kernel(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *Ipub,
                                  const int *pub2int, int grid_limit, hipStream_t st) {
    const int n = tp.n;
    if (n > 0) {
        // grid_limit > 0: a persistent grid of that size striding over the items
        int *ticket = grid_limit > 0 ? nullptr : tp.ticket;
        const bool mixed = rc.prec == COIL_MIXED;
        const int grid = grid_limit > 0 ? min(grid_limit, n)
                         : ticket       ? queue_grid(mixed ? tp.grid32 : tp.grid64, n)
                                        : n;
        if (mixed)
            hipLaunchKernelGGL(k_field_tz32, dim3(grid), dim3(64), 0, st, s, rc, tp.items, tp.rows, n,
                               static_cast<const float *>(tp.Ipub32), pub2int, ticket);
        else
            hipLaunchKernelGGL(k_field_tz64, dim3(grid), dim3(64), 0, st, s, rc, tp.items, tp.rows, n, Ipub,
                               pub2int, ticket);
    }
    return hipGetLastError();
}

hipError_t launch_flux_tz(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *vpub,
                          const int *pub2int, const int *done, hipStream_t st) {
    const int n = tp.n;
    if (n > 0)
        hipLaunchKernelGGL(k_flux_tz64, dim3(queue_grid(tp.gridF64, n)), dim3(64), 0, st, s, rc, tp.items, tp.rows,
                           n, vpub, pub2int, tp.ticket, done);
    return hipGetLastError();
}

hipError_t launch_fieldT_tz(const DevState &s, const RunConst &rc, const TzPlan &tp, const double *wr,
                            const double *wz, double *wr_pub, double *wz_pub, const int *pub2int,
                            double *partT, hipStream_t st) {
    int *ticket = tp.ticket ? tp.ticket + 1 : nullptr;
    hipLaunchKernelGGL(k_to_pub, dim3((s.N + 255) / 256), dim3(256), 0, st, wr, s.perm, s.N, wr_pub, ticket,
                       static_cast<float *>(nullptr), s.elem_coil, s.coils);
    hipLaunchKernelGGL(k_to_pub, dim3((s.N + 255) / 256), dim3(256), 0, st, wz, s.perm, s.N, wz_pub,
                       static_cast<int *>(nullptr), static_cast<float *>(nullptr), s.elem_coil, s.coils);
    const int n = tp.n;
    if (n > 0) {
        const bool mixed = rc.prec == COIL_MIXED;
        const int grid = ticket ? queue_grid(mixed ? tp.gridT32 : tp.gridT64, n) : n;
        if (mixed)
            hipLaunchKernelGGL(k_fieldT_tz32, dim3(grid), dim3(64), 0, st, s, rc, tp.items, tp.rows, n, wr_pub,
                               wz_pub, pub2int, partT, ticket);
        else
            hipLaunchKernelGGL(k_fieldT_tz64, dim3(grid), dim3(64), 0, st, s, rc, tp.items, tp.rows, n, wr_pub,
                               wz_pub, pub2int, partT, ticket);
    }
    return hipGetLastError();
}

}  // namespace coilq
