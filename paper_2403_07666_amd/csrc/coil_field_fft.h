// coil_field_fft.h -- field pass by fast convolution (coil_field_fft.hip).
//
// On a coil's regular (r, z) grid the all-pairs field sum is, for every pair
// of rows (target row i, source row j), a 1-D linear convolution along z of
// the source currents with g(i, j, delta), delta = z_target - z_source in
// [-(Z-1), Z-1].  Zero-padded to a length L >= 2Z - 1 (a power of two) the
// linear convolution equals the circular one, so with the DFT over z
//   B^_i[f] = sum_j G^_ij[f] I^_j[f]   for each of the L/2 + 1 bins f,
// and B_i = inverse DFT of B^_i on the first Z points.  The spectra G^ of the
// kernel values are made once at set-up (FP64 Green's function, FP64 DFT;
// stored in FP32 in mixed precision, the pass's other arithmetic is FP64);
// g_z is even in delta, so G^_z is real, g_r is odd, so G^_r = i S with S
// real: two real R x R matrices per bin.  A pass is then
//   1. the forward transform of the source rows (two rows per complex DFT),
//   2. per bin, the two real matrices times the complex vector of the rows
//      (the whole pass streams the spectra once: HBM-bound),
//   3. the inverse transform of each target row (B_z + i B_r in one DFT).
// Every pair (e, j) still contributes g(e, j) I_j exactly once; the sum is
// the same as the pairwise passes' up to rounding.  The transposed pass (the
// adjoint's) uses the same spectra with conj(G^).
#pragma once

#include <vector>

#include "coil_internal.h"

namespace coilq {

constexpr int kFftMaxLog = 12;    // L <= 4096 (n_z <= 2048)
constexpr int kFftJ = 256;        // bin products: source rows per workgroup (64 per wave)
constexpr int kFftI = 256;        // bin products: target rows per workgroup (4 per lane, 64 lanes)

struct FftCoil {
    int R, Rp, Z, L, logL, bins;  // rows, rows padded to 4, row length, DFT length, log2 L, L/2 + 1
    int P;                        // forward bin products: source-row parts (partials) of kFftJ
    int IB;                       // transposed bin products: target blocks (partials) of kFftI
    int off;                      // first element of the coil
    int sym;                      // S kept as its packed upper triangle (FP64, one block: n_r <= 256)
    double kscale;                // mu0 / (2 pi d)
    double kflux;                 // mu0 d: the flux kernel's scale
    double c2d;                   // 2 r_inner / d + 1 (grid units)
    size_t spec;   // offset (reals) of the coil's G^_z; S follows after bins R Rp
    size_t sp;     // sym: reals of one bin's packed S (sym_row(R)); S[f] at spec + bins R Rp + f sp
    size_t fspec;  // offset (FP64 reals) of its flux spectra M^[f][j][i] (coupled solve)
    size_t hat;    // offset (reals) of its transformed rows: bins Rp 4 reals
    size_t bpart;  // offset (reals) of its partial bin products
};

// Packed upper triangle of a symmetric n x n matrix by rows: row j holds
// columns 0 .. j, padded with zeros to a multiple of 4 (4 ceil((j + 1) / 4)
// reals); sym_row(j) is its offset, sym_row(n) the size (about n^2 / 2).
__host__ __device__ inline size_t sym_row(int j) {
    const size_t q = (size_t)j >> 2, r = (size_t)j & 3;
    return 4 * (q + 1) * (2 * q + r);
}

struct FftPlan {
    const FftCoil *coils;
    // [pairs | rows | bins (coils without sym) | binsT (same) | sym bins (coil, f) | bins of every coil (flux)]
    const int4 *items;
    int npairs, nrows, nbins, nbinsT, nsym, nflux;
    int Lmax, logLmax;
    int prec;           // COIL_MIXED: spectra stored in FP32; COIL_FP64: in FP64
    void *spec;
    double *fspec;      // flux spectra (FP64; null unless the coupled solve uses this pass)
    double *hat, *bpart;
    const double2 *tw64;  // exp(-2 pi i k / Lmax), k < Lmax / 2
};

// host plan of one coil set: per-coil records, items and sizes (in reals)
struct FftHostPlan {
    std::vector<FftCoil> coils;
    std::vector<int4> items;
    int npairs = 0, nrows = 0, nbins = 0, nbinsT = 0, nsym = 0, nflux = 0;
    int Lmax = 2, logLmax = 1;
    int flux = 0;  // also the flux kernel's spectra
    size_t spec_reals = 0, hat_reals = 0, bpart_reals = 0;  // spectra in their precision, others FP64
    size_t flux_reals = 0;
};

// the plan for coils of (layers * ne) x (turns * ne) grids (flux: also the
// spectra of the mutual-inductance kernel, for the coupled solve)
void fft_plan(const std::vector<CoilDev> &coils, int flux, int prec, FftHostPlan &fp);

// the spectra of every coil (FP64 DFT of the FP64 kernel values), stored in
// the pass's precision; tmp: staging of tmp_bytes bytes (a slab of source rows)
hipError_t launch_fft_setup(const DevState &s, const FftPlan &fp, const FftCoil *host_coils, int ncoils,
                            void *tmp, size_t tmp_bytes, hipStream_t st);

// forward pass: part[0][e] = (sum g_r I, sum g_z I) with I = kscale * s.I
hipError_t launch_field_fft(const DevState &s, const FftPlan &fp, const int *pub2int, hipStream_t st);

// flux pass of the coupled solve: part[0][e] = (0, sum_j M(e, j) v_j) with M
// the mutual inductance of the rings of e and j (none for j = e), v in
// internal order; every kernel returns at once when *done != 0
hipError_t launch_flux_fft(const DevState &s, const FftPlan &fp, const double *v, const int *pub2int,
                           const int *done, hipStream_t st);

// transposed pass: partT[0][j] = sum_e [ wr_e g_r(e, j) + wz_e g_z(e, j) ]
hipError_t launch_fieldT_fft(const DevState &s, const FftPlan &fp, const double *wr, const double *wz,
                             const int *pub2int, double *partT, hipStream_t st);

}  // namespace coilq
