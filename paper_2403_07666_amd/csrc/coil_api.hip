// coil_api.hip -- host side of the C ABI declared in include/coil.h:
// validation, device layout planning, precompute (geometry, per-layer
// inductance blocks, heat conductances, bounding boxes, field-pass work
// items), step sequencing, HIP event timing and HIP graph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "coil_adjoint.h"
#include "coil_coupled.h"
#include "coil_field_fft.h"
#include "coil_field_tz.h"
#include "coil_internal.h"

using namespace coilq;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHECK(x)                                                                       \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail(COIL_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *coil_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ plan
namespace {

struct Buf {  // one carved region
    size_t off, bytes;
};

struct Plan {
    int N = 0, Nw = 0, nlayers = 0, ngroups = 0, nsub = 1, max_ne2 = 1, nheat_blocks = 0, nrows = 0;
    int tile_targets = 256;
    std::vector<CoilDev> coils;
    std::vector<PairItem> items;
    int nchunk_max = 1;
    size_t items_cap = 0;  // work-item capacity (autotuner candidates)
    std::vector<TzItem> tz_items;  // translation-reuse pass, longest items first
    std::vector<int> tz_rows;      // per coil, its source rows in bit-reversed order
    int nslot_tz_max = 1;
    int part_slots = 2;  // capacity of part[] in double2 slots of N
    double tz_evals = 0.0;  // kernel-value evaluations of one translation-reuse pass
    size_t tz_cap = 0;      // translation item capacity (kTzMaxSplit source-row groups)
    std::vector<int2> near_pair;  // mixed mode: per coil, per (target row, source row): (first, count)
    size_t near_total = 0;        // near kernel values over all pairs
    int algo = COIL_ALGO_TRANSLATION;
    int fft = 0;            // COIL_ALGO_FFT at init: the spectra and buffers of the fast-convolution pass
    FftHostPlan fftp;
    int prec = COIL_FP64;  // arithmetic of the field passes (sets the width choice)
    int coupled = 0;       // COIL_COUPLE_FULL: buffers of the coupled solve
    int adi = 0;           // COIL_HEAT_ADI: buffers of the ADI heat step
    int nsubel = 0;        // subelement model: subelements per wire side (0 = off)
    int em = 0;            // variable-step EM integration
    std::vector<int> fast_w0;  // fast wire kernel: first wire of each workgroup (up to kFastWires of one layer)
    int ncols = 0, hb_slots = 1, maxline = 0;
    int nchunk_cap = 1;    // partial-sum capacity in chunks
    size_t total = 0;
    // regions
    Buf coils_b, items_b, bbox_b, gpos_b, rho_b, r_b, V_b, invV_b, jcs_b, psi_b, G_b, Gb_b, nb_b,
        perm_b, wire_coil_b, fastw_b, elem_coil_b, Mlay_b, Minv_b, yl_b, syl_b, wflag_b, cw_b, I_b, Phi_b, Br_b, Bz_b, E_b, Ep_b, dI_b,
        q_b, Jc_b, u_b[3], T_b[3], part_b, Uw_b, Qw_b, wq_b, wmaxx_b, hb_max_b, hb_arg_b, hb_out_b,
        sc_b, tmp_b, misc_b, diag_b, hrow_b, Lself_b, cgv_b, cgL_b, cgred_b, cgrw_b, cgsc_b, adi_b, kmult_b, IH_b, emsub_b, tz_b, tzrows_b, Ipub_b, pub2int_b, zphys_b, near_pair_b, near_val_b, ticket_b,
        Ipub32_b, fftspec_b, ffthat_b, fftbp_b, fftitems_b, fftcoils_b, ffttw64_b, fftflux_b;
};

Buf carve(size_t &cur, size_t bytes) {
    cur = (cur + 255) & ~size_t(255);
    Buf b{cur, bytes};
    cur += bytes;
    return b;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const coil_config *c) {
    if (!c) return fail(COIL_E_INVAL, "config is NULL");
    if (c->n_coils < 1 || c->n_coils > 4096) return fail(COIL_E_INVAL, "n_coils out of range");
    if (!c->layers || !c->turns || !c->ne || !c->r_inner || !c->z_center || !c->wire_side || !c->ramp)
        return fail(COIL_E_INVAL, "per-coil array is NULL");
    long long N = 0;
    for (int i = 0; i < c->n_coils; ++i) {
        if (c->layers[i] < 1 || c->turns[i] < 1 || c->ne[i] < 1)
            return fail(COIL_E_INVAL, "coil %d: layers, turns and ne must be >= 1", i);
        if (c->ne[i] * c->ne[i] > kMaxWireElems)
            return fail(COIL_E_INVAL, "coil %d: ne^2 = %d exceeds %d elements per wire", i,
                        c->ne[i] * c->ne[i], kMaxWireElems);
        const long long nr = (long long)c->layers[i] * c->ne[i], nz = (long long)c->turns[i] * c->ne[i];
        if (nr > 2048 || nz > 2048)
            return fail(COIL_E_INVAL, "coil %d: grid %lld x %lld exceeds 2048 per side", i, nr, nz);
        if (!finite_pos(c->r_inner[i]) || !finite_pos(c->wire_side[i]) || !std::isfinite(c->z_center[i]) ||
            !std::isfinite(c->ramp[i]))
            return fail(COIL_E_INVAL, "coil %d: bad geometry or ramp", i);
        N += nr * nz;
    }
    if (N > (1LL << 30)) return fail(COIL_E_INVAL, "too many elements");
    if (!finite_pos(c->dt) || !finite_pos(c->Ec) || !(std::isfinite(c->n) && c->n >= 1.0) ||
        !finite_pos(c->Jc0) || !finite_pos(c->Tc) || !finite_pos(c->B0) || !finite_pos(c->C0) ||
        !finite_pos(c->T_ref) || !finite_pos(c->k0) || !(std::isfinite(c->h0) && c->h0 >= 0.0) ||
        !finite_pos(c->T_bath) || !(std::isfinite(c->cp_exp) && c->cp_exp >= 0.0) ||
        !std::isfinite(c->dBa_dt) || !(std::isfinite(c->eps_coef) && std::isfinite(c->eps_pow)))
        return fail(COIL_E_INVAL, "material or time-step constant out of range");
    if (c->precision != COIL_FP64 && c->precision != COIL_MIXED)
        return fail(COIL_E_INVAL, "unknown precision %d", c->precision);
    if (!(c->near_k == 0.0 || (c->near_k > 0.0 && c->near_k < 1.0)))
        return fail(COIL_E_INVAL, "near_k must be in (0, 1) or 0");
    if (c->heat_substeps < 0 || c->heat_substeps > 100000) return fail(COIL_E_INVAL, "heat_substeps out of range");
    if (!(c->tile_targets == 0 || c->tile_targets == 64 || c->tile_targets == 128 || c->tile_targets == 256))
        return fail(COIL_E_INVAL, "tile_targets must be 0, 64, 128 or 256");
    if (c->tile_sources < 0 || c->tile_sources % kStage != 0)
        return fail(COIL_E_INVAL, "tile_sources must be a non-negative multiple of %d", kStage);
    if (c->grid_limit < 0) return fail(COIL_E_INVAL, "grid_limit must be >= 0");
    if (c->algo < COIL_ALGO_AUTO || c->algo > COIL_ALGO_FFT) return fail(COIL_E_INVAL, "unknown algo %d", c->algo);
    if (c->I0)
        for (int i = 0; i < c->n_coils; ++i)
            if (!std::isfinite(c->I0[i])) return fail(COIL_E_INVAL, "coil %d: non-finite I0", i);
    if (!(std::isfinite(c->rho_n) && c->rho_n >= 0.0)) return fail(COIL_E_INVAL, "rho_n must be finite and >= 0");
    if (c->geometry != COIL_AXISYMMETRIC && c->geometry != COIL_PLANAR)
        return fail(COIL_E_INVAL, "unknown geometry %d", c->geometry);
    if (c->coupling != COIL_COUPLE_TRANSPORT && c->coupling != COIL_COUPLE_FULL)
        return fail(COIL_E_INVAL, "unknown coupling %d", c->coupling);
    if (c->heat_solver != COIL_HEAT_EXPLICIT && c->heat_solver != COIL_HEAT_ADI)
        return fail(COIL_E_INVAL, "unknown heat_solver %d", c->heat_solver);
    if (c->heat_solver == COIL_HEAT_ADI)
        for (int i = 0; i < c->n_coils; ++i)
            if ((long long)c->layers[i] * c->ne[i] > 1536 || (long long)c->turns[i] * c->ne[i] > 1536)
                return fail(COIL_E_INVAL, "coil %d: the ADI heat step takes at most 1536 elements per grid side", i);
    if (!(std::isfinite(c->ins_R0) && c->ins_R0 >= 0.0)) return fail(COIL_E_INVAL, "ins_R0 must be finite and >= 0");
    if (c->ins_R0 != 0.0 && c->heat_solver != COIL_HEAT_ADI)
        return fail(COIL_E_INVAL, "an insulation resistance (ins_R0) needs heat_solver = COIL_HEAT_ADI");
    if (!std::isfinite(c->k_exp) || !std::isfinite(c->h_exp))
        return fail(COIL_E_INVAL, "k_exp and h_exp must be finite");
    if ((c->k_exp != 0.0 || c->h_exp != 0.0) && c->heat_solver != COIL_HEAT_ADI)
        return fail(COIL_E_INVAL, "temperature-dependent k or h (k_exp, h_exp) needs heat_solver = COIL_HEAT_ADI");
    if (c->cg_max_iter < 0 || !(std::isfinite(c->cg_tol) && c->cg_tol >= 0.0))
        return fail(COIL_E_INVAL, "cg_max_iter must be >= 0 and cg_tol finite and >= 0");
    if (!(std::isfinite(c->em_tol) && c->em_tol >= 0.0) || c->em_max_level < 0 || c->em_max_level > 16)
        return fail(COIL_E_INVAL, "em_tol must be finite and >= 0, em_max_level in 0 .. 16");
    if (c->em_tol > 0.0 && (c->coupling != COIL_COUPLE_TRANSPORT || c->subelements != 0))
        return fail(COIL_E_INVAL, "the variable step (em_tol > 0) takes the wire model with transport-only coupling");
    if (c->subelements < 0 || c->subelements > kMaxSubelements)
        return fail(COIL_E_INVAL, "subelements must be in 0 .. %d", kMaxSubelements);
    if (c->subelements > 0) {
        for (int i = 0; i < c->n_coils; ++i)
            if (c->ne[i] % c->subelements != 0)
                return fail(COIL_E_INVAL, "coil %d: ne = %d is not a multiple of subelements = %d", i, c->ne[i],
                            c->subelements);
        if (c->coupling == COIL_COUPLE_FULL)
            return fail(COIL_E_INVAL, "the subelement model takes the transport-only coupling");
    }
    return COIL_OK;
}

constexpr int kMaxChunks = 16;

// ---- field-pass work plans (begin)
// Field-pass work items: targets in blocks of tb, sources of each coil in
// chunks.  nch_req > 0 asks for that many chunks per coil, cs_req > 0 for a
// chunk size; both 0: enough chunks for >= ~2048 items in total.  Chunks are
// multiples of the LDS stage.
void build_items(Plan &p, int tb, int nch_req, int cs_req) {
    p.items.clear();
    p.tile_targets = tb;
    p.nchunk_max = 1;
    long long total_blocks = 0;
    for (auto &d : p.coils) total_blocks += (d.n + tb - 1) / tb;
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        CoilDev &d = p.coils[ci];
        int cs = cs_req;
        if (cs == 0) {
            const long long want = nch_req > 0 ? nch_req
                                               : std::max<long long>(1, (2048 + total_blocks - 1) / total_blocks);
            const long long maxch = (d.n + kStage - 1) / kStage;
            const long long ch = std::min(want, maxch);
            cs = (int)(((d.n + ch - 1) / ch + kStage - 1) / kStage * kStage);
        }
        d.nchunk = (d.n + cs - 1) / cs;
        p.nchunk_max = std::max(p.nchunk_max, d.nchunk);
        for (int t0 = 0; t0 < d.n; t0 += tb)
            for (int k = 0; k < d.nchunk; ++k) {
                PairItem it;
                it.coil = (int)ci;
                it.t0 = d.off + t0;
                it.tn = std::min(tb, d.n - t0);
                it.s0 = d.off + k * cs;
                it.sn = std::min(cs, d.n - k * cs);
                it.chunk = k;
                p.items.push_back(it);
            }
    }
}

// Translation-reuse work items: target row segments of 64 W (W = 2 .. 8
// targets per thread) x source-row groups.  Each coil's rows are cut into the
// segment widths that minimise the estimated time, sum over segments of
// 64 W / eff(W), where eff(W) is the measured relative throughput per target
// slot of width W on this GPU, per precision (single coils of 64 layers and
// 128 W turns-elements; the window holds 2W accumulators per LDS read, and
// every width runs at the register count of the widest).
// The source rows of a target segment are split into n_g groups: enough for
// about 8192 items (four or more per LDS slot of the GPU), and more for large
// coils, so that an item of the largest coil holds at most about 4e6 pairs
// (the end of the pass, where SIMDs run out of items at different times,
// scales with the item); at most kTzMaxSplit.  A group is a run of
// the coil's rows in bit-reversed order, so that it samples the whole coil
// (a like share of near rows), and the group sizes fall linearly from 4 to 1
// relative units.  All items run in one launch, the most FMA work first, so the
// last items dispatched are the shortest and the end of the pass, where a SIMD
// is left with a single wave, is short.
constexpr int kTzMaxSplit = 64;

// m1 below which the mixed field passes evaluate the kernel in FP64 (k near 1)
float m1_near_of(const coil_config *c) {
    const double nk = c->near_k > 0.0 ? c->near_k : 0.99;
    return (float)(1.0 - nk * nk);
}

// Near kernel values of the mixed translation pass.  For a pair of rows
// (a, b) of a coil, m1 = al2 / be2 grows with delta^2, so m1 < m1_near holds
// exactly for delta^2 < (m1_near sr^2 - dr^2) / (1 - m1_near) (dr = a - b,
// sr = c2d + a + b): |delta| < count.  count is capped at the largest |delta|
// any table of the coil can hold (n_z + 1024).
bool build_near(Plan &p, float m1_near) {
    p.near_pair.clear();
    p.near_total = 0;
    for (CoilDev &d : p.coils) {
        d.near_base = (int)p.near_pair.size();
        if (p.prec != COIL_MIXED) continue;
        const int nr = d.layers * d.ne, nz = d.turns * d.ne;
        const double m = m1_near;
        const long long amax = (long long)nz + 1024;
        for (int a = 0; a < nr; ++a)
            for (int b = 0; b < nr; ++b) {
                const double dr = (double)(a - b), sr = d.c2d + (double)(a + b);
                const double t = (m * sr * sr - dr * dr) / (1.0 - m);
                long long cnt = 0;
                if (t > 0.0) {
                    long long r = (long long)std::sqrt(t);  // largest r with r^2 < t
                    while (r > 0 && (double)(r * r) >= t) --r;
                    while ((double)((r + 1) * (r + 1)) < t) ++r;
                    cnt = std::min(r, amax) + 1;
                }
                if (p.near_total + (size_t)cnt > (size_t)INT_MAX) return false;  // int2 offsets
                p.near_pair.push_back(make_int2((int)p.near_total, (int)cnt));
                p.near_total += (size_t)cnt;
            }
    }
    return true;
}

std::vector<int> group_sizes(int nr, int ns) {
    std::vector<int> sz(ns, 1);
    if (ns <= 1) {
        sz.assign(1, nr);
        return sz;
    }
    std::vector<double> wgt(ns);
    double tot = 0.0;
    for (int g = 0; g < ns; ++g) tot += (wgt[g] = 4.0 - 3.0 * g / (ns - 1));
    int used = 0;
    for (int g = 0; g < ns; ++g) used += (sz[g] = std::max(1, (int)std::floor(wgt[g] / tot * nr)));
    for (int g = 0; used < nr; g = (g + 1) % ns, ++used) ++sz[g];  // remainder to the first groups
    for (int g = ns - 1; used > nr; g = g > 0 ? g - 1 : ns - 1)
        if (sz[g] > 1) --sz[g], --used;
    return sz;
}

void build_tz(Plan &p, int nsplit_req, int force_w = 0) {
    static const double eff64[kTzNW] = {0.41, 0.52, 0.71, 0.78, 0.84, 0.91, 1.0};
    static const double eff32[kTzNW] = {0.29, 0.45, 0.63, 0.74, 0.84, 0.91, 1.0};
    const double *eff = p.prec == COIL_MIXED ? eff32 : eff64;
    std::vector<TzItem> items;
    std::vector<std::vector<int>> segw(p.coils.size());  // width index per segment
    long long segs = 0;
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        const CoilDev &d = p.coils[ci];
        const int nz = d.turns * d.ne, nr = d.layers * d.ne;
        std::vector<double> cost(nz + 1, 0.0);
        std::vector<int> pick(nz + 1, 0);
        for (int rem = 1; rem <= nz; ++rem) {
            cost[rem] = INFINITY;
            for (int wi = 0; wi < kTzNW; ++wi) {
                const int span = 64 * (wi + 2);
                const double c = span / eff[wi] + cost[std::max(0, rem - span)];
                if (c < cost[rem]) {
                    cost[rem] = c;
                    pick[rem] = wi;
                }
            }
        }
        if (force_w >= 2 && force_w <= 8) {  // one width for every segment
            for (int z0 = 0; z0 < nz; z0 += 64 * force_w) segw[ci].push_back(force_w - 2);
        } else {
            for (int z0 = 0; z0 < nz; z0 += 64 * (pick[nz - z0] + 2)) segw[ci].push_back(pick[nz - z0]);
        }
        segs += (long long)nr * (long long)segw[ci].size();
    }
    // the split is common to all coils: the largest coil's items set the size bound
    long long by_size = 1;
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        const CoilDev &d = p.coils[ci];
        const double csegs = (double)d.layers * d.ne * (double)segw[ci].size();
        by_size = std::max(by_size, (long long)std::ceil((double)d.n * (double)(d.n - 1) / (csegs * 4e6)));
    }
    const long long by_count = (8192 + segs - 1) / segs;
    const int nsplit = nsplit_req > 0 ? std::min(nsplit_req, kTzMaxSplit)
                                      : (int)std::max<long long>(1, std::min<long long>(kTzMaxSplit, std::max(by_count, by_size)));
    p.nslot_tz_max = 1;
    p.tz_evals = 0.0;
    p.tz_rows.clear();
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        CoilDev &d = p.coils[ci];
        const int nz = d.turns * d.ne, nr = d.layers * d.ne;
        const int ns = std::min(nsplit, nr);
        d.nslot_tz = ns;
        p.nslot_tz_max = std::max(p.nslot_tz_max, ns);
        // rows in bit-reversed order (ties, from rows past a power of two, by row)
        const int base = (int)p.tz_rows.size();
        int bits = 0;
        while ((1 << bits) < nr) ++bits;
        std::vector<std::pair<unsigned, int>> key(nr);
        for (int r = 0; r < nr; ++r) {
            unsigned v = 0;
            for (int b = 0; b < bits; ++b) v |= ((unsigned)(r >> b) & 1u) << (bits - 1 - b);
            key[r] = {v, r};
        }
        std::sort(key.begin(), key.end());
        for (const auto &kv : key) p.tz_rows.push_back(kv.second);
        const std::vector<int> gsz = group_sizes(nr, ns);
        int z0 = 0;
        for (int wi : segw[ci]) {
            const int W = wi + 2;
            for (int ir = 0; ir < nr; ++ir)
                for (int g = 0, start = 0; g < ns; start += gsz[g], ++g) {
                    TzItem it{};
                    it.coil = (int)ci;
                    it.ir = ir;
                    it.z0 = z0;
                    it.roff = base + start;
                    it.rcnt = gsz[g];
                    it.slot = g;
                    it.w = W;
                    items.push_back(it);
                }
            // kernel-value evaluations per pass: for a chunk of se sources the
            // forward table holds 64 W + se entries at delta = dlo + tau,
            // dlo = z0 - s0 - se; an entry is evaluated unless delta < 0 and its
            // mirror -delta is in the table
            const int smax = W >= 5 ? 512 : 256;
            for (int s0 = 0; s0 < nz; s0 += smax) {
                const int se = (std::min(smax, nz - s0) + W - 1) / W * W;
                const int nt = 64 * W + se, dlo = z0 - s0 - se;
                // evaluated: tau >= -dlo (delta >= 0), or tau < -dlo with -2 dlo - tau >= nt
                const long long pos = std::max(0, nt - std::max(0, -dlo));
                const long long neg_far = std::max(0, std::min(-dlo, -2 * dlo - nt + 1));
                p.tz_evals += (double)nr * (double)nr * (double)(pos + std::max(0LL, std::min(neg_far, (long long)nt)));
                if (p.prec == COIL_MIXED && !p.near_pair.empty()) {
                    // near entries come from the set-up table: not evaluated per pass
                    const long long p0 = std::max(dlo, 0), p1 = (long long)dlo + nt;  // delta >= 0 evaluated
                    const long long q0 = std::max(1LL, (long long)dlo + nt), q1 = -(long long)dlo;  // |delta| of negatives
                    long long look = 0;
                    for (int pr = 0; pr < nr * nr; ++pr) {
                        const long long cnt = p.near_pair[d.near_base + pr].y;
                        look += std::max(0LL, std::min(p1, cnt) - p0);
                        look += std::max(0LL, std::min(q1, cnt - 1) - q0 + 1);
                    }
                    p.tz_evals -= (double)look;
                }
            }
            z0 += 64 * W;
        }
    }
    // one launch, the most FMA work (targets x source rows x sources) first
    auto work = [&](const TzItem &it) {
        const CoilDev &d = p.coils[it.coil];
        return (long long)it.w * it.rcnt * (long long)(d.turns * d.ne);
    };
    std::stable_sort(items.begin(), items.end(), [&](const TzItem &a, const TzItem &b) { return work(a) > work(b); });
    p.tz_items = std::move(items);
}
// ---- field-pass work plans (end)

int make_plan(const coil_config *c, Plan &p) {
    p = Plan();
    p.prec = c->precision;
    p.coupled = c->coupling == COIL_COUPLE_FULL ? 1 : 0;
    p.adi = c->heat_solver == COIL_HEAT_ADI ? 1 : 0;
    p.nsubel = c->subelements;
    p.em = c->em_tol > 0.0 ? 1 : 0;
    int off = 0, woff = 0, loff = 0, goff = 0, toff = 0, roff = 0;
    for (int i = 0; i < c->n_coils; ++i) {
        CoilDev d{};
        d.ne = c->ne[i];
        d.ne2 = d.ne * d.ne;
        d.layers = c->layers[i];
        d.turns = c->turns[i];
        d.n = d.layers * d.turns * d.ne2;
        d.off = off;
        d.wire_off = woff;
        d.layer_off = loff;
        d.group_off = goff;
        d.d = c->wire_side[i] / d.ne;
        const double rho0 = c->r_inner[i] / d.d;
        d.c2d = 2.0 * rho0 + 1.0;
        d.c2f = (float)d.c2d;
        d.kscale = kMu0 / (2.0 * kPi * d.d);
        d.dIt = c->ramp[i] * c->dt;
        d.I0e = (c->I0 ? c->I0[i] : 0.0) / d.ne2;
        d.tile_off = toff;
        d.ntile_z = (d.turns * d.ne + kHT - 1) / kHT;
        d.row_off = roff;
        d.col_off = p.ncols;
        toff += (d.layers * d.ne + kHT - 1) / kHT * d.ntile_z;
        roff += d.layers * d.ne;
        p.ncols += d.turns * d.ne;
        p.maxline = std::max(p.maxline, std::max(d.layers * d.ne, d.turns * d.ne));
        off += d.n;
        woff += d.layers * d.turns;
        loff += d.layers;
        goff += (d.n + kGroup - 1) / kGroup;
        p.max_ne2 = std::max(p.max_ne2, d.ne2);
        for (int l = 0; l < d.layers; ++l)
            for (int t = 0; t < d.turns; t += kFastWires) p.fast_w0.push_back(d.wire_off + l * d.turns + t);
        p.coils.push_back(d);
    }
    p.N = off;
    p.Nw = woff;
    p.nlayers = loff;
    p.ngroups = goff;
    p.nheat_blocks = p.adi ? std::max(p.ncols, roff) : toff;
    p.nrows = roff;
    int tb = c->tile_targets;
    if (tb == 0) tb = p.N <= 8192 ? 64 : 256;
    if (!build_near(p, m1_near_of(c))) return fail(COIL_E_INVAL, "near-value table exceeds 2^31 entries");
    build_items(p, tb, 0, c->tile_sources);
    // capacity for the autotuner's candidates: targets per item >= 64 and at
    // most kMaxChunks source chunks per coil
    Plan q = p;
    size_t cap = p.items.size();
    int pcap = p.nchunk_max;
    for (int t : {64, 128, 256})
        for (int ch : {1, 2, 4, 8, kMaxChunks}) {
            build_items(q, t, ch, 0);
            cap = std::max(cap, q.items.size());
            pcap = std::max(pcap, q.nchunk_max);
        }
    p.items_cap = cap;
    p.nchunk_cap = pcap;
    for (int fw : {0, 2, 3, 4, 5, 6, 7, 8}) {  // capacity for every split and forced width
        Plan q = p;
        build_tz(q, kTzMaxSplit, fw);
        p.tz_cap = std::max(p.tz_cap, q.tz_items.size());
        p.nchunk_cap = std::max(p.nchunk_cap, q.nslot_tz_max);
    }
    build_tz(p, 0);
    p.tz_cap = std::max(p.tz_cap, p.tz_items.size());
    p.algo = c->algo == COIL_ALGO_DIRECT ? COIL_ALGO_DIRECT : COIL_ALGO_TRANSLATION;
    if (c->algo == COIL_ALGO_FFT) {
        p.algo = COIL_ALGO_FFT;
        p.fft = 1;
        fft_plan(p.coils, p.coupled, p.prec, p.fftp);
    }
    return COIL_OK;
}

int heat_substeps(const coil_config *c, const Plan &p) {
    if (c->heat_solver == COIL_HEAT_ADI) return 1;  // one implicit step
    if (c->heat_substeps > 0) return c->heat_substeps;
    // explicit stability limit at T_bath: h_max = min_e V_e C(T_bath) / (sum of
    // the element's face and border conductances)
    const double Cb = c->C0 * std::pow(c->T_bath / c->T_ref, c->cp_exp);
    double hmax = INFINITY;
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        const CoilDev &d = p.coils[ci];
        const int nr = d.layers * d.ne, nz = d.turns * d.ne;
        const double rin = c->r_inner[ci];
        const bool planar = c->geometry == COIL_PLANAR;
        for (int ir = 0; ir < nr; ++ir) {
            const double re = rin + (ir + 0.5) * d.d;
            const double V = planar ? d.d * d.d : 2.0 * kPi * re * d.d * d.d;
            double faces[4] = {2.0 * kPi * (rin + ir * d.d) * d.d, 2.0 * kPi * (rin + (ir + 1) * d.d) * d.d,
                               2.0 * kPi * re * d.d, 2.0 * kPi * re * d.d};
            if (planar) faces[0] = faces[1] = faces[2] = faces[3] = d.d;
            for (int iz = 0; iz < nz; ++iz) {
                const bool has[4] = {ir > 0, ir < nr - 1, iz > 0, iz < nz - 1};
                double g = 0.0;
                for (int f = 0; f < 4; ++f) {
                    if (has[f]) g += c->k0 * faces[f] / d.d;
                    else if (c->h0 > 0.0) g += faces[f] / (1.0 / c->h0 + d.d / (2.0 * c->k0));
                }
                if (g > 0.0) hmax = std::min(hmax, V * Cb / g);
            }
        }
    }
    const double qt = c->dt / (0.9 * hmax);
    const long ns = (long)std::ceil(qt * (1.0 - 1.0e-9));
    return (int)std::max(1L, ns);
}

size_t layout(Plan &p) {
    size_t cur = 0;
    const size_t N = p.N, Nw = p.Nw, d8 = sizeof(double);
    p.coils_b = carve(cur, sizeof(CoilDev) * p.coils.size());
    p.items_b = carve(cur, sizeof(PairItem) * std::max<size_t>(1, std::max(p.items.size(), p.items_cap)));
    p.bbox_b = carve(cur, sizeof(int4) * std::max(1, p.ngroups));
    p.gpos_b = carve(cur, sizeof(float2) * N);
    p.rho_b = carve(cur, d8 * N);
    p.r_b = carve(cur, d8 * N);
    p.V_b = carve(cur, d8 * N);
    p.invV_b = carve(cur, d8 * N);
    p.jcs_b = carve(cur, d8 * N);
    p.psi_b = carve(cur, d8 * N);
    p.G_b = carve(cur, d8 * 4 * N);
    p.Gb_b = carve(cur, d8 * N);
    p.nb_b = carve(cur, sizeof(int) * 4 * N);
    p.perm_b = carve(cur, sizeof(int) * N);
    p.wire_coil_b = carve(cur, sizeof(int) * Nw);
    p.fastw_b = carve(cur, sizeof(int) * p.fast_w0.size());
    p.elem_coil_b = carve(cur, sizeof(int) * N);
    size_t mlay = 0;
    for (auto &d : p.coils) mlay += (size_t)d.layers * d.ne2 * d.ne2;
    p.Mlay_b = carve(cur, d8 * mlay);
    p.Minv_b = carve(cur, d8 * mlay);
    size_t ylen = 0;
    for (auto &d : p.coils) ylen += (size_t)d.layers * d.ne2;
    p.yl_b = carve(cur, d8 * ylen);
    p.syl_b = carve(cur, d8 * p.nlayers);
    p.wflag_b = carve(cur, sizeof(int) * Nw);
    p.cw_b = carve(cur, d8 * Nw);
    p.I_b = carve(cur, d8 * N);
    p.Phi_b = carve(cur, d8 * N);
    p.Br_b = carve(cur, d8 * N);
    p.Bz_b = carve(cur, d8 * N);
    p.E_b = carve(cur, d8 * N);
    p.Ep_b = carve(cur, d8 * N);
    p.dI_b = carve(cur, d8 * N);
    p.q_b = carve(cur, d8 * N);
    p.Jc_b = carve(cur, d8 * N);
    for (int i = 0; i < 3; ++i) {
        p.u_b[i] = carve(cur, d8 * N);
        p.T_b[i] = carve(cur, d8 * N);
    }
    // partial sums: every tiling's slot count, and at least 2 slots so that the
    // transposed test hook can stage 2N doubles after N partials
    p.part_slots = std::max({p.nchunk_max, p.nchunk_cap, p.nslot_tz_max, 2});
    p.part_b = carve(cur, sizeof(double2) * N * p.part_slots);
    p.tz_b = carve(cur, sizeof(TzItem) * std::max<size_t>(1, std::max(p.tz_items.size(), p.tz_cap)));
    p.tzrows_b = carve(cur, sizeof(int) * std::max<size_t>(1, p.tz_rows.size()));
    p.Ipub_b = carve(cur, sizeof(double) * N);
    p.Ipub32_b = carve(cur, sizeof(float) * N);
    p.pub2int_b = carve(cur, sizeof(int) * N);
    p.zphys_b = carve(cur, sizeof(double) * N);
    p.near_pair_b = carve(cur, sizeof(int2) * std::max<size_t>(1, p.near_pair.size()));
    p.near_val_b = carve(cur, sizeof(float2) * std::max<size_t>(1, p.near_total));
    p.ticket_b = carve(cur, 2 * sizeof(int));
    p.Uw_b = carve(cur, d8 * Nw);
    p.Qw_b = carve(cur, d8 * Nw);
    p.wq_b = carve(cur, d8 * Nw);
    p.wmaxx_b = carve(cur, d8 * Nw);
    p.diag_b = carve(cur, d8 * 6 * Nw);
    p.hrow_b = carve(cur, sizeof(HeatRow) * std::max(1, p.nrows));
    p.hb_max_b = carve(cur, d8 * p.nheat_blocks);
    p.hb_arg_b = carve(cur, sizeof(long long) * p.nheat_blocks);
    p.hb_slots = p.adi ? 2 : p.nsub;
    p.hb_out_b = carve(cur, d8 * (size_t)p.nheat_blocks * p.hb_slots);
    p.sc_b = carve(cur, sizeof(Scalars));
    p.tmp_b = carve(cur, d8 * std::max<size_t>(N, Nw));
    p.misc_b = carve(cur, d8 * 64);
    if (p.adi) {
        p.adi_b = carve(cur, d8 * 10 * N);  // Cv, G (4), Gbr, Gbz, Lz0, Lr1, Ts
        p.kmult_b = carve(cur, d8 * N);
    }
    if (p.nsubel) p.IH_b = carve(cur, d8 * N);
    if (p.em) p.emsub_b = carve(cur, d8 * Nw);
    if (p.fft) {
        const size_t rs = p.prec == COIL_MIXED ? sizeof(float) : sizeof(double);
        p.fftspec_b = carve(cur, rs * p.fftp.spec_reals);
        p.ffthat_b = carve(cur, d8 * p.fftp.hat_reals);
        p.fftbp_b = carve(cur, d8 * p.fftp.bpart_reals);
        p.fftitems_b = carve(cur, sizeof(int4) * p.fftp.items.size());
        p.fftflux_b = carve(cur, d8 * std::max<size_t>(1, p.fftp.flux_reals));
        p.fftcoils_b = carve(cur, sizeof(FftCoil) * p.fftp.coils.size());
        p.ffttw64_b = carve(cur, sizeof(double2) * (p.fftp.Lmax / 2));
    }
    if (p.coupled) {
        p.Lself_b = carve(cur, d8 * N);
        p.cgv_b = carve(cur, d8 * 5 * N);
        p.cgL_b = carve(cur, d8 * Nw * (size_t)packed_size(p.max_ne2));
        p.cgred_b = carve(cur, d8 * ((N + 255) / 256));
        p.cgrw_b = carve(cur, d8 * 2 * Nw);
        p.cgsc_b = carve(cur, sizeof(CgScalars));
    }
    p.total = (cur + 255) & ~size_t(255);
    return p.total;
}

}  // namespace

namespace {
int scratch_for_current_device(double2 **out);  // defined with the static scratch below
}  // namespace

// ------------------------------------------------------------------ handle
struct coil_s {
    Plan plan;
    RunConst rc{};
    DevState ds{};
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    int grid_limit = 0;
    double T_bath = 4.2;
    std::vector<double> r_pub, z_pub;  // public order, for COIL_F_R / COIL_F_Z
    std::vector<int> pub2int;          // public -> internal element index
    TzPlan tz{};                       // device items of the translation-reuse pass
    FftPlan fft{};                     // device plan of the fast-convolution pass (COIL_ALGO_FFT at init)
    double *Ipub = nullptr;            // currents in public order (its input)
    int *d_pub2int = nullptr;
    // timing
    bool timing = false;
    bool timing_all = false;  // all phases, or only the field kernel
    struct Pending {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    double ms[4] = {0, 0, 0, 0};
    long long launches[4] = {0, 0, 0, 0};
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    long long gsteps = 0;
    bool capturing = false;
    int tz_split = 0;    // source-row groups of the translation pass (0 = automatic)
    int tz_force_w = 0;  // segment width of the translation pass (0 = automatic)
    double2 *scratch = nullptr;  // this device's static scratch (coil_field_at_noalloc)
    double cg_tol = 1e-12;       // coupled solve: relative residual to reach
    int cg_maxit = 100;          // coupled solve: iterations per step at most
    int cg_check = 8;            // eager stepping: iterations between convergence checks
    // coil_run: the heat step and reductions of step k on a second stream, so
    // that they overlap the field pass of step k + 1 (which reads only I)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool side_pending = false;  // side-stream work not yet joined into `stream`
};

namespace {

template <typename T>
T *at(coil_t *h, const Buf &b) {
    return reinterpret_cast<T *>(h->ws + b.off);
}

int ev_get(coil_t *h, hipEvent_t *e) {
    if (!h->pool.empty()) {
        *e = h->pool.back();
        h->pool.pop_back();
        return COIL_OK;
    }
    HIPCHECK(hipEventCreate(e));
    return COIL_OK;
}

int t_begin(coil_t *h, hipEvent_t *a, int phase) {
    if (!h->timing || (phase != 0 && !h->timing_all)) return COIL_OK;
    int rc = ev_get(h, a);
    if (rc) return rc;
    HIPCHECK(hipEventRecord(*a, h->stream));
    return COIL_OK;
}

int t_end(coil_t *h, int phase, hipEvent_t a, int nlaunch) {
    if (!h->timing || (phase != 0 && !h->timing_all)) return COIL_OK;
    hipEvent_t b;
    int rc = ev_get(h, &b);
    if (rc) return rc;
    HIPCHECK(hipEventRecord(b, h->stream));
    h->pending.push_back({phase, a, b});
    h->launches[phase] += nlaunch;
    return COIL_OK;
}

int t_flush(coil_t *h) {
    if (h->pending.empty()) return COIL_OK;
    HIPCHECK(hipStreamSynchronize(h->stream));
    for (auto &p : h->pending) {
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, p.a, p.b));
        h->ms[p.phase] += ms;
        h->pool.push_back(p.a);
        h->pool.push_back(p.b);
    }
    h->pending.clear();
    return COIL_OK;
}

// transposed field pass into partT, by the handle's algorithm; wpub: 2N doubles
hipError_t launch_fieldT_any(coil_t *h, const double *wr, const double *wz, double *wpub, double *partT,
                             hipStream_t st) {
    const DevState &d = h->ds;
    if (d.algo_fft) return launch_fieldT_fft(d, h->fft, wr, wz, h->d_pub2int, partT, st);
    if (d.algo_tz)
        return launch_fieldT_tz(d, h->rc, h->tz, wr, wz, wpub, wpub + d.N, h->d_pub2int, partT, st);
    return launch_fieldT(d, h->rc, h->grid_limit, wr, wz, partT, st);
}

hipError_t launch_field_any(coil_t *h, const DevState &d, hipStream_t st) {
    if (d.algo_fft) return launch_field_fft(d, h->fft, h->d_pub2int, st);
    if (d.algo_tz) return launch_field_tz(d, h->rc, h->tz, h->Ipub, h->d_pub2int, h->grid_limit, st);
    return launch_field(d, h->rc, h->grid_limit, st);
}

// The coupled A-V solve after the deferred per-wire kernels.  Eager stepping
// reads the convergence flag every cg_check iterations (a host
// synchronisation); under graph capture all cg_maxit iterations are enqueued
// and those after convergence return at once.
int coupled_solve(coil_t *h) {
    const DevState &d = h->ds;
    HIPCHECK(launch_cg_begin(d, h->rc, h->tz, h->fft, h->Ipub, h->d_pub2int, h->cg_tol, h->cg_maxit, h->stream));
    for (int it = 0; it < h->cg_maxit; ++it) {
        HIPCHECK(launch_cg_iteration(d, h->rc, h->tz, h->fft, h->Ipub, h->d_pub2int, h->stream));
        if (!h->capturing && (it + 1) % h->cg_check == 0 && it + 1 < h->cg_maxit) {
            int done = 0;
            HIPCHECK(hipMemcpyAsync(&done, &d.cg->done, sizeof(int), hipMemcpyDeviceToHost, h->stream));
            HIPCHECK(hipStreamSynchronize(h->stream));
            if (done) break;
        }
    }
    HIPCHECK(launch_cg_finish(d, h->rc, h->stream));
    return COIL_OK;
}

// the side stream's work of the last overlapped step into the handle's stream
int join_side(coil_t *h) {
    if (!h->side_pending) return COIL_OK;
    HIPCHECK(hipStreamWaitEvent(h->stream, h->ev_join, 0));
    h->side_pending = false;
    return COIL_OK;
}

// One step.  overlap: the heat step and the reductions go to the side stream
// after the wire phase, and the next step's wire phase waits for them (it
// reads T and rewrites the per-wire sums they reduce); the next field pass
// does not, it reads only the currents.  The caller joins the side stream
// (join_side) before anything else reads the state.  Only under the
// fast-convolution pass, whose kernels leave room on the CUs: the
// translation pass fills every CU with as many work-queue workgroups as fit,
// and a concurrent heat kernel's workgroups then hold slots its late
// workgroups wait for (measured at C2: 1267 -> 1072 steps/s, against
// 8711 -> 9842 under the fast convolution).
int enqueue_step(coil_t *h, bool overlap = false) {
    hipEvent_t a = nullptr;
    int rc;
    // phase 0 brackets the field kernel alone (its input reordering runs before)
    const DevState &d = h->ds;
    if (d.algo_tz) HIPCHECK(launch_field_tz_prep(d, h->tz, h->Ipub, h->stream));
    if ((rc = t_begin(h, &a, 0))) return rc;
    if (d.algo_fft)
        HIPCHECK(launch_field_fft(d, h->fft, h->d_pub2int, h->stream));
    else if (d.algo_tz)
        HIPCHECK(launch_field_tz_kernel(d, h->rc, h->tz, h->Ipub, h->d_pub2int, h->grid_limit, h->stream));
    else
        HIPCHECK(launch_field(d, h->rc, h->grid_limit, h->stream));
    if ((rc = t_end(h, 0, a, 1))) return rc;
    if ((rc = join_side(h))) return rc;
    if ((rc = t_begin(h, &a, 1))) return rc;
    HIPCHECK(launch_wire(h->ds, h->rc, h->stream));
    if (d.cg_defer && (rc = coupled_solve(h))) return rc;
    if ((rc = t_end(h, 1, a, 1))) return rc;
    overlap = overlap && h->side && d.algo_fft && !(h->timing && h->timing_all);
    if (overlap) {
        HIPCHECK(hipEventRecord(h->ev_fork, h->stream));
        HIPCHECK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
        HIPCHECK(launch_heat_step(h->ds, h->rc, h->side));
        HIPCHECK(launch_finalize(h->ds, h->rc, h->side));
        HIPCHECK(hipEventRecord(h->ev_join, h->side));
        h->side_pending = true;
        if (h->timing && h->pending.size() > 16384) return t_flush(h);
        return COIL_OK;
    }
    if ((rc = t_begin(h, &a, 2))) return rc;
    HIPCHECK(launch_heat_step(h->ds, h->rc, h->stream));
    if ((rc = t_end(h, 2, a, h->rc.adi ? 3 : heat_launches(h->ds.nsub)))) return rc;
    if ((rc = t_begin(h, &a, 3))) return rc;
    HIPCHECK(launch_finalize(h->ds, h->rc, h->stream));
    if ((rc = t_end(h, 3, a, 1))) return rc;
    if (h->timing && h->pending.size() > 16384) return t_flush(h);
    return COIL_OK;
}

int reset_state(coil_t *h) {
    const DevState &s = h->ds;
    hipStream_t st = h->stream;
    HIPCHECK(launch_init_current(s, st));
    HIPCHECK(launch_fill(s.Phi, 0.0, s.N, st));
    HIPCHECK(launch_fill(s.Br, 0.0, s.N, st));
    HIPCHECK(launch_fill(s.Bz, 0.0, s.N, st));
    HIPCHECK(launch_fill(s.E, 0.0, s.N, st));
    HIPCHECK(launch_fill(s.Ep, 0.0, s.N, st));
    HIPCHECK(launch_fill(s.dI, 0.0, s.N, st));
    HIPCHECK(launch_fill(s.q, 0.0, s.N, st));
    HIPCHECK(launch_fill(s.Jc, 0.0, s.N, st));
    for (int i = 0; i < 3; ++i) {
        HIPCHECK(launch_fill(s.u[i], 0.0, s.N, st));
        HIPCHECK(launch_fill(s.T[i], h->T_bath, s.N, st));
    }
    HIPCHECK(launch_fill(reinterpret_cast<double *>(s.part), 0.0, 2 * s.N * h->plan.part_slots, st));
    HIPCHECK(launch_fill(s.Uw, 0.0, s.Nw, st));
    HIPCHECK(launch_zero_int(s.wflag, s.Nw, st));
    HIPCHECK(launch_fill(s.Qw, 0.0, s.Nw, st));
    HIPCHECK(launch_fill(s.wq, 0.0, s.Nw, st));
    HIPCHECK(launch_fill(s.wmaxx, 0.0, s.Nw, st));
    HIPCHECK(launch_fill(s.onset, -1.0, 2 * s.Nw, st));  // onset and quench
    HIPCHECK(launch_fill(s.Qon, 0.0, 4 * s.Nw, st));     // Qon, Qqu, Tqu, Pqu
    if (s.IH) HIPCHECK(launch_fill(s.IH, 0.0, s.N, st));
    if (s.emsub) HIPCHECK(launch_fill(s.emsub, 0.0, s.Nw, st));
    if (s.cg) HIPCHECK(launch_fill(reinterpret_cast<double *>(s.cg), 0.0, sizeof(CgScalars) / sizeof(double), st));
    HIPCHECK(launch_reset_scalars(s.sc, h->T_bath, st));
    return COIL_OK;
}

}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" int coil_query(const coil_config *cfg, coil_sizes *out) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!out) return fail(COIL_E_INVAL, "out is NULL");
    Plan p;
    if ((rc = make_plan(cfg, p))) return rc;
    p.nsub = heat_substeps(cfg, p);
    layout(p);
    out->workspace_bytes = p.total;
    out->n_elem = p.N;
    out->n_wire = p.Nw;
    out->heat_substeps = p.nsub;
    out->n_work_items = (int32_t)p.items.size();
    return COIL_OK;
}

extern "C" int coil_init(const coil_config *cfg, const coil_inputs *in, void *workspace,
                         size_t workspace_bytes, void *stream, coil_t **out) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!out) return fail(COIL_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!workspace) return fail(COIL_E_INVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(COIL_E_INVAL, "workspace must be 256-byte aligned");
    coil_t *h = new (std::nothrow) coil_t();
    if (!h) return fail(COIL_E_NOMEM, "host allocation failed");
    std::unique_ptr<coil_t, void (*)(coil_t *)> guard(h, [](coil_t *p) { coil_destroy(p); });
    Plan &p = h->plan;
    if ((rc = make_plan(cfg, p))) return rc;
    p.nsub = heat_substeps(cfg, p);
    layout(p);
    if (workspace_bytes < p.total)
        return fail(COIL_E_NOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes,
                    p.total);
    h->ws = static_cast<char *>(workspace);
    h->stream = static_cast<hipStream_t>(stream);
    if (h->stream) {  // side stream (default priority) and its fork/join events
        HIPCHECK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    }
    h->grid_limit = cfg->grid_limit;
    h->T_bath = cfg->T_bath;
    const int N = p.N, Nw = p.Nw;

    // run constants
    RunConst &r = h->rc;
    r.Ec = cfg->Ec;
    r.n = cfg->n;
    r.Tc = cfg->Tc;
    r.B0 = cfg->B0;
    r.dt = cfg->dt;
    r.dBa_dt = cfg->dBa_dt;
    r.T_bath = cfg->T_bath;
    r.T_ref = cfg->T_ref;
    r.C0 = cfg->C0;
    r.cp_exp = cfg->cp_exp;
    const double p1 = cfg->cp_exp + 1.0;
    r.u_a1 = p1 / (cfg->C0 * cfg->T_ref);
    r.u_a0 = std::pow(cfg->T_bath / cfg->T_ref, p1);
    r.u_inv = 1.0 / p1;
    r.m1_near = m1_near_of(cfg);
    r.prec = cfg->precision;
    r.rho_n = cfg->rho_n;
    r.k0 = cfg->k0;
    r.h0 = cfg->h0;
    r.k_exp = cfg->k_exp;
    r.h_exp = cfg->h_exp;
    r.ins_R0 = cfg->ins_R0;
    r.adi = p.adi;
    r.em_tol = cfg->em_tol;
    r.em_levels = cfg->em_max_level > 0 ? cfg->em_max_level : 10;
    const bool planar = cfg->geometry == COIL_PLANAR;

    // host precompute, internal (wire-major) order
    std::vector<float2> gpos(N);
    std::vector<double> zphys(N);
    std::vector<double> rho(N), rr(N), V(N), invV(N), jcs(N), G(4 * (size_t)N), Gb(N);
    std::vector<int> nb(4 * (size_t)N), perm(N), wire_coil(Nw), elem_coil(N);
    std::vector<int4> bbox(std::max(1, p.ngroups));
    std::vector<double> Mlay;
    std::vector<int> pub2int(N);
    h->r_pub.assign(N, 0.0);
    h->z_pub.assign(N, 0.0);
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        const CoilDev &d = p.coils[ci];
        const int ne = d.ne, nz = d.turns * ne;
        const double rin = cfg->r_inner[ci];
        const double zbot = cfg->z_center[ci] - 0.5 * d.turns * cfg->wire_side[ci];
        for (int L = 0; L < d.layers; ++L)
            for (int Tn = 0; Tn < d.turns; ++Tn) {
                const int w = d.wire_off + L * d.turns + Tn;
                wire_coil[w] = (int)ci;
                for (int a = 0; a < ne; ++a)
                    for (int b = 0; b < ne; ++b) {
                        const int e = d.off + (L * d.turns + Tn) * d.ne2 + a * ne + b;
                        const int ir = L * ne + a, iz = Tn * ne + b;
                        const int pub = d.off + ir * nz + iz;
                        perm[e] = pub;
                        pub2int[pub] = e;
                        elem_coil[e] = (int)ci;
                        gpos[e] = make_float2((float)ir, (float)iz);
                        rho[e] = rin / d.d + ir + 0.5;
                        rr[e] = rin + (ir + 0.5) * d.d;
                        V[e] = planar ? d.d * d.d : 2.0 * kPi * rr[e] * d.d * d.d;
                        invV[e] = 1.0 / V[e];
                        h->r_pub[pub] = rr[e];
                        h->z_pub[pub] = zbot + (iz + 0.5) * d.d;
                        zphys[e] = h->z_pub[pub];
                    }
            }
    }
    // Jc static part and per-wire multiplier
    std::vector<double> cw(Nw, 1.0);
    for (int e = 0; e < N; ++e) {
        const int pub = perm[e];
        const double mu = (in && in->jc0_mult) ? in->jc0_mult[pub] : 1.0;
        const double ep = (in && in->strain) ? in->strain[pub] : 0.0;
        jcs[e] = cfg->Jc0 * mu * (1.0 - cfg->eps_coef * std::pow(std::fabs(ep), cfg->eps_pow));
        if (!std::isfinite(jcs[e])) return fail(COIL_E_INVAL, "non-finite Jc0 multiplier or strain at %d", pub);
    }
    std::vector<double> kmult(p.adi ? N : 0, 1.0);
    if (in && in->k_mult) {
        for (int e = 0; e < N; ++e) {
            const double v = in->k_mult[perm[e]];
            if (!(std::isfinite(v) && v > 0.0)) return fail(COIL_E_INVAL, "k_mult must be finite and > 0 (element %d)", perm[e]);
            if (v != 1.0 && !p.adi) return fail(COIL_E_INVAL, "a conductivity map (k_mult) needs heat_solver = COIL_HEAT_ADI");
            if (p.adi) kmult[e] = v;
        }
    }
    if (in && in->c_wire)
        for (int w = 0; w < Nw; ++w) {
            cw[w] = in->c_wire[w];
            if (!std::isfinite(cw[w])) return fail(COIL_E_INVAL, "non-finite c_wire at %d", w);
        }
    // heat conductances (axisymmetric finite volumes)
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        const CoilDev &d = p.coils[ci];
        const int ne = d.ne, nr = d.layers * ne, nz = d.turns * ne;
        const double rin = cfg->r_inner[ci];
        for (int ir = 0; ir < nr; ++ir)
            for (int iz = 0; iz < nz; ++iz) {
                const int pub = d.off + ir * nz + iz;
                const int e = pub2int[pub];
                const double re = rin + (ir + 0.5) * d.d;
                double area[4] = {2.0 * kPi * (rin + ir * d.d) * d.d, 2.0 * kPi * (rin + (ir + 1) * d.d) * d.d,
                                  2.0 * kPi * re * d.d, 2.0 * kPi * re * d.d};
                if (planar) area[0] = area[1] = area[2] = area[3] = d.d;
                const int nbp[4] = {ir > 0 ? pub - nz : -1, ir < nr - 1 ? pub + nz : -1, iz > 0 ? pub - 1 : -1,
                                    iz < nz - 1 ? pub + 1 : -1};
                double gb = 0.0;
                for (int f = 0; f < 4; ++f) {
                    if (nbp[f] >= 0) {
                        nb[4 * (size_t)e + f] = pub2int[nbp[f]];
                        G[4 * (size_t)e + f] = cfg->k0 * area[f] / d.d;
                    } else {
                        nb[4 * (size_t)e + f] = -1;
                        G[4 * (size_t)e + f] = 0.0;
                        if (cfg->h0 > 0.0) gb += area[f] / (1.0 / cfg->h0 + d.d / (2.0 * cfg->k0));
                    }
                }
                Gb[e] = gb;
            }
    }
    // the same conductances per grid row, for the tiled heat step (identical
    // expressions, so the values are bitwise those of G, Gb and invV above)
    std::vector<HeatRow> hrow(std::max(1, p.nrows));
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        const CoilDev &d = p.coils[ci];
        const int nr = d.layers * d.ne;
        const double rin = cfg->r_inner[ci];
        for (int ir = 0; ir < nr; ++ir) {
            const double re = rin + (ir + 0.5) * d.d;
            double area[4] = {2.0 * kPi * (rin + ir * d.d) * d.d, 2.0 * kPi * (rin + (ir + 1) * d.d) * d.d,
                              2.0 * kPi * re * d.d, 2.0 * kPi * re * d.d};
            if (planar) area[0] = area[1] = area[2] = area[3] = d.d;
            const double Ve = planar ? d.d * d.d : 2.0 * kPi * re * d.d * d.d;
            HeatRow R{};
            R.ain = area[0];
            R.aout = area[1];
            R.aax = area[2];
            R.gin = cfg->k0 * area[0] / d.d;
            R.gout = cfg->k0 * area[1] / d.d;
            R.gax = cfg->k0 * area[2] / d.d;
            R.invV = 1.0 / Ve;
            if (cfg->h0 > 0.0) {
                R.gbin = area[0] / (1.0 / cfg->h0 + d.d / (2.0 * cfg->k0));
                R.gbout = area[1] / (1.0 / cfg->h0 + d.d / (2.0 * cfg->k0));
                R.gbax = area[2] / (1.0 / cfg->h0 + d.d / (2.0 * cfg->k0));
            }
            hrow[d.row_off + ir] = R;
        }
    }
    // bounding boxes of 64-element groups (grid indices)
    for (const CoilDev &d : p.coils)
        for (int g = 0; g < (d.n + kGroup - 1) / kGroup; ++g) {
            int4 bb = make_int4(1 << 30, -(1 << 30), 1 << 30, -(1 << 30));
            for (int e = d.off + g * kGroup; e < std::min(d.off + d.n, d.off + (g + 1) * kGroup); ++e) {
                const int ir = (int)gpos[e].x, iz = (int)gpos[e].y;
                bb.x = std::min(bb.x, ir);
                bb.y = std::max(bb.y, ir);
                bb.z = std::min(bb.z, iz);
                bb.w = std::max(bb.w, iz);
            }
            bbox[d.group_off + g] = bb;
        }
    // per-layer inductance blocks (column-major), grid units
    for (size_t ci = 0; ci < p.coils.size(); ++ci) {
        const CoilDev &d = p.coils[ci];
        const int ne = d.ne, n = d.ne2;
        const double rho0 = cfg->r_inner[ci] / d.d;
        for (int L = 0; L < d.layers; ++L) {
            const size_t base = Mlay.size();
            Mlay.resize(base + (size_t)n * n);
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int ai = i / ne, bi = i % ne, aj = j / ne, bj = j % ne;
                    const double ri = rho0 + L * ne + ai + 0.5, rj = rho0 + L * ne + aj + 0.5;
                    double m;
                    if (i == j) {
                        m = kMu0 * ri * d.d * (std::log(8.0 * ri / kGmdSquare) - 2.0);
                    } else {
                        const double dr = (double)(ai - aj), dz = (double)(bi - bj);
                        const double sr = ri + rj;
                        const double al2 = dr * dr + dz * dz, be2 = sr * sr + dz * dz;
                        const double m1 = al2 / be2;
                        double K, E;
                        host_ellip_f64(m1, &K, &E);
                        m = kMu0 * std::sqrt(be2) * d.d * (0.5 * (1.0 + m1) * K - E);
                    }
                    Mlay[base + (size_t)j * n + i] = m;
                }
        }
    }

    // per-layer inverse, M^-1 1 and its sum (Cholesky on the host, FP64)
    std::vector<double> Minv(Mlay.size()), yl, syl;
    {
        size_t base = 0;
        for (const CoilDev &d : p.coils) {
            const int n = d.ne2;
            for (int L = 0; L < d.layers; ++L, base += (size_t)n * n) {
                std::vector<double> Lf(Mlay.begin() + base, Mlay.begin() + base + (size_t)n * n);
                // column-major lower Cholesky in place: Lf[j*n + i], i >= j
                for (int j = 0; j < n; ++j) {
                    double djj = Lf[(size_t)j * n + j];
                    for (int k = 0; k < j; ++k) djj -= Lf[(size_t)k * n + j] * Lf[(size_t)k * n + j];
                    if (!(djj > 0.0)) return fail(COIL_E_NONFINITE, "inductance block of layer %d is not positive definite", L);
                    const double ljj = std::sqrt(djj);
                    Lf[(size_t)j * n + j] = ljj;
                    for (int i = j + 1; i < n; ++i) {
                        double v = Lf[(size_t)j * n + i];
                        for (int k = 0; k < j; ++k) v -= Lf[(size_t)k * n + i] * Lf[(size_t)k * n + j];
                        Lf[(size_t)j * n + i] = v / ljj;
                    }
                }
                std::vector<double> col(n);
                double ssum = 0.0;
                for (int c = 0; c < n; ++c) {
                    for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
                    for (int i = 0; i < n; ++i) {
                        double v = col[i];
                        for (int k = 0; k < i; ++k) v -= Lf[(size_t)k * n + i] * col[k];
                        col[i] = v / Lf[(size_t)i * n + i];
                    }
                    for (int i = n - 1; i >= 0; --i) {
                        double v = col[i];
                        for (int k = i + 1; k < n; ++k) v -= Lf[(size_t)i * n + k] * col[k];
                        col[i] = v / Lf[(size_t)i * n + i];
                    }
                    for (int i = 0; i < n; ++i) Minv[base + (size_t)c * n + i] = col[i];
                }
                for (int i = 0; i < n; ++i) {
                    double v = 0.0;
                    for (int c = 0; c < n; ++c) v += Minv[base + (size_t)c * n + i];
                    yl.push_back(v);
                    ssum += v;
                }
                syl.push_back(ssum);
            }
        }
    }

    // device pointers
    DevState &s = h->ds;
    s.N = N;
    s.Nw = Nw;
    s.ngroups = p.ngroups;
    s.nitems = (int)p.items.size();
    s.nheat_blocks = p.nheat_blocks;
    s.ncoils = (int)p.coils.size();
    s.hrow = at<HeatRow>(h, p.hrow_b);
    s.hb_slots = p.hb_slots;
    if (p.adi) {
        double *a = at<double>(h, p.adi_b);
        s.adi_Cv = a;
        s.adi_G = a + N;
        s.adi_Gbr = a + 5 * (size_t)N;
        s.adi_Gbz = a + 6 * (size_t)N;
        s.adi_Lz0 = a + 7 * (size_t)N;
        s.adi_Lr1 = a + 8 * (size_t)N;
        s.adi_Ts = a + 9 * (size_t)N;
        s.kmult = at<double>(h, p.kmult_b);
        s.adi_ncols = p.ncols;
        s.adi_nrows = p.nrows;
        s.adi_maxline = p.maxline;
    }
    s.nsub = p.nsub;
    s.max_ne2 = p.max_ne2;
    s.tile_targets = p.tile_targets;
    s.algo_tz = p.algo == COIL_ALGO_TRANSLATION ? 1 : 0;
    s.algo_fft = p.algo == COIL_ALGO_FFT ? 1 : 0;
    s.flux_fft = p.fft && p.fftp.flux ? 1 : 0;
    if (p.fft) {
        FftPlan &f = h->fft;
        f.coils = at<FftCoil>(h, p.fftcoils_b);
        f.items = at<int4>(h, p.fftitems_b);
        f.npairs = p.fftp.npairs;
        f.nrows = p.fftp.nrows;
        f.nbins = p.fftp.nbins;
        f.nbinsT = p.fftp.nbinsT;
        f.nsym = p.fftp.nsym;
        f.nflux = p.fftp.nflux;
        f.Lmax = p.fftp.Lmax;
        f.logLmax = p.fftp.logLmax;
        f.prec = p.prec;
        f.spec = at<char>(h, p.fftspec_b);
        f.fspec = p.fftp.flux ? at<double>(h, p.fftflux_b) : nullptr;
        f.hat = at<double>(h, p.ffthat_b);
        f.bpart = at<double>(h, p.fftbp_b);
        f.tw64 = at<double2>(h, p.ffttw64_b);
    }
    h->Ipub = at<double>(h, p.Ipub_b);
    h->d_pub2int = at<int>(h, p.pub2int_b);
    h->tz.items = at<TzItem>(h, p.tz_b);
    h->tz.rows = at<int>(h, p.tzrows_b);
    h->tz.n = (int)p.tz_items.size();
    h->tz.ticket = at<int>(h, p.ticket_b);
    h->tz.Ipub32 = p.prec == COIL_MIXED ? at<float>(h, p.Ipub32_b) : nullptr;
    HIPCHECK(tz_resident_grids(h->tz));
    if ((rc = scratch_for_current_device(&h->scratch))) return rc;
    s.coils = at<CoilDev>(h, p.coils_b);
    s.items = at<PairItem>(h, p.items_b);
    s.bbox = at<int4>(h, p.bbox_b);
    s.gpos = at<float2>(h, p.gpos_b);
    s.rho = at<double>(h, p.rho_b);
    s.r = at<double>(h, p.r_b);
    s.V = at<double>(h, p.V_b);
    s.invV = at<double>(h, p.invV_b);
    s.jcs = at<double>(h, p.jcs_b);
    s.psi = at<double>(h, p.psi_b);
    s.G = at<double>(h, p.G_b);
    s.Gb = at<double>(h, p.Gb_b);
    s.nb = at<int>(h, p.nb_b);
    s.perm = at<int>(h, p.perm_b);
    s.wire_coil = at<int>(h, p.wire_coil_b);
    s.fast_w0 = at<int>(h, p.fastw_b);
    s.nfast = (int)p.fast_w0.size();
    s.elem_coil = at<int>(h, p.elem_coil_b);
    s.Mlay = at<double>(h, p.Mlay_b);
    s.Minv = at<double>(h, p.Minv_b);
    s.yl = at<double>(h, p.yl_b);
    s.syl = at<double>(h, p.syl_b);
    s.wflag = at<int>(h, p.wflag_b);
    s.cw = at<double>(h, p.cw_b);
    s.I = at<double>(h, p.I_b);
    s.Phi = at<double>(h, p.Phi_b);
    s.Br = at<double>(h, p.Br_b);
    s.Bz = at<double>(h, p.Bz_b);
    s.E = at<double>(h, p.E_b);
    s.Ep = at<double>(h, p.Ep_b);
    s.dI = at<double>(h, p.dI_b);
    s.q = at<double>(h, p.q_b);
    s.Jc = at<double>(h, p.Jc_b);
    for (int i = 0; i < 3; ++i) {
        s.u[i] = at<double>(h, p.u_b[i]);
        s.T[i] = at<double>(h, p.T_b[i]);
    }
    s.part = at<double2>(h, p.part_b);
    s.near_pair = at<int2>(h, p.near_pair_b);
    s.near_val = at<float2>(h, p.near_val_b);
    s.Uw = at<double>(h, p.Uw_b);
    s.Qw = at<double>(h, p.Qw_b);
    s.wq = at<double>(h, p.wq_b);
    s.wmaxx = at<double>(h, p.wmaxx_b);
    {
        double *dg = at<double>(h, p.diag_b);
        s.onset = dg;
        s.quench = dg + Nw;
        s.Qon = dg + 2 * (size_t)Nw;
        s.Qqu = dg + 3 * (size_t)Nw;
        s.Tqu = dg + 4 * (size_t)Nw;
        s.Pqu = dg + 5 * (size_t)Nw;
    }
    s.hb_max = at<double>(h, p.hb_max_b);
    s.hb_arg = at<long long>(h, p.hb_arg_b);
    s.hb_out = at<double>(h, p.hb_out_b);
    s.sc = at<Scalars>(h, p.sc_b);
    if (p.nsubel) {
        s.nsubel = p.nsubel;
        s.IH = at<double>(h, p.IH_b);
    }
    if (p.em) s.emsub = at<double>(h, p.emsub_b);
    if (p.coupled) {
        s.cg_defer = 1;
        s.Lself = at<double>(h, p.Lself_b);
        double *v = at<double>(h, p.cgv_b);
        s.cg_x = v;
        s.cg_r = v + N;
        s.cg_z = v + 2 * (size_t)N;
        s.cg_p = v + 3 * (size_t)N;
        s.cg_q = v + 4 * (size_t)N;
        s.cg_L = at<double>(h, p.cgL_b);
        s.cg_red = at<double>(h, p.cgred_b);
        s.cg_rw = at<double>(h, p.cgrw_b);
        s.cg_cw = s.cg_rw + Nw;
        s.cg = at<CgScalars>(h, p.cgsc_b);
        h->cg_tol = cfg->cg_tol > 0.0 ? cfg->cg_tol : 1e-12;
        h->cg_maxit = cfg->cg_max_iter > 0 ? cfg->cg_max_iter : 100;
    }
    s.tmp = at<double>(h, p.tmp_b);

    hipStream_t st = h->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    HIPCHECK(up((void *)s.coils, p.coils.data(), sizeof(CoilDev) * p.coils.size()));
    HIPCHECK(up((void *)s.items, p.items.data(), sizeof(PairItem) * p.items.size()));
    HIPCHECK(up((void *)s.bbox, bbox.data(), sizeof(int4) * p.ngroups));
    HIPCHECK(up((void *)s.gpos, gpos.data(), sizeof(float2) * N));
    HIPCHECK(up((void *)s.rho, rho.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.r, rr.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.V, V.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.invV, invV.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.jcs, jcs.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.G, G.data(), sizeof(double) * 4 * N));
    HIPCHECK(up((void *)s.Gb, Gb.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.hrow, hrow.data(), sizeof(HeatRow) * p.nrows));
    if (p.adi) HIPCHECK(up((void *)s.kmult, kmult.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.nb, nb.data(), sizeof(int) * 4 * N));
    HIPCHECK(up((void *)s.perm, perm.data(), sizeof(int) * N));
    HIPCHECK(up((void *)s.wire_coil, wire_coil.data(), sizeof(int) * Nw));
    HIPCHECK(up((void *)s.fast_w0, p.fast_w0.data(), sizeof(int) * p.fast_w0.size()));
    HIPCHECK(up((void *)s.elem_coil, elem_coil.data(), sizeof(int) * N));
    HIPCHECK(up((void *)s.Mlay, Mlay.data(), sizeof(double) * Mlay.size()));
    HIPCHECK(up((void *)s.Minv, Minv.data(), sizeof(double) * Minv.size()));
    HIPCHECK(up((void *)s.yl, yl.data(), sizeof(double) * yl.size()));
    HIPCHECK(up((void *)s.syl, syl.data(), sizeof(double) * syl.size()));
    std::vector<double> Lself;
    if (p.coupled) {  // the self inductances, as on the diagonals of the layer blocks
        Lself.resize(N);
        size_t base = 0;
        for (const CoilDev &d : p.coils) {
            const int n = d.ne2;
            for (int w = 0; w < d.layers * d.turns; ++w)
                for (int i = 0; i < n; ++i)
                    Lself[d.off + (size_t)w * n + i] = Mlay[base + (size_t)(w / d.turns) * n * n + (size_t)i * n + i];
            base += (size_t)d.layers * n * n;
        }
        HIPCHECK(up((void *)s.Lself, Lself.data(), sizeof(double) * N));
    }
    HIPCHECK(up((void *)s.cw, cw.data(), sizeof(double) * Nw));
    HIPCHECK(up((void *)h->tz.items, p.tz_items.data(), sizeof(TzItem) * p.tz_items.size()));
    HIPCHECK(up((void *)h->tz.rows, p.tz_rows.data(), sizeof(int) * p.tz_rows.size()));
    HIPCHECK(up((void *)h->d_pub2int, pub2int.data(), sizeof(int) * N));
    HIPCHECK(up((void *)at<double>(h, p.zphys_b), zphys.data(), sizeof(double) * N));
    HIPCHECK(up((void *)s.near_pair, p.near_pair.data(), sizeof(int2) * p.near_pair.size()));
    HIPCHECK(hipMemsetAsync(h->tz.ticket, 0, 2 * sizeof(int), st));
    if (p.prec == COIL_MIXED)
        for (size_t ci = 0; ci < p.coils.size(); ++ci)
            HIPCHECK(launch_near_fill(s, (int)ci, p.coils[ci].layers * p.coils[ci].ne, st));
    std::vector<double2> tw64;
    if (p.fft) {  // twiddles exp(-2 pi i k / Lmax), then the spectra
        const int Lm = p.fftp.Lmax;
        tw64.resize(Lm / 2);
        for (int k = 0; k < Lm / 2; ++k) {
            const double th = 2.0 * kPi * (double)k / (double)Lm;
            tw64[k] = make_double2(std::cos(th), -std::sin(th));
        }
        HIPCHECK(up((void *)h->fft.tw64, tw64.data(), sizeof(double2) * tw64.size()));
        HIPCHECK(up((void *)h->fft.coils, p.fftp.coils.data(), sizeof(FftCoil) * p.fftp.coils.size()));
        HIPCHECK(up((void *)h->fft.items, p.fftp.items.data(), sizeof(int4) * p.fftp.items.size()));
        // staging: the partial-sum buffer (a slab of source rows at a time)
        HIPCHECK(launch_fft_setup(s, h->fft, p.fftp.coils.data(), (int)p.fftp.coils.size(), s.part,
                                  sizeof(double2) * (size_t)N * p.part_slots, st));
    }
    // transport-flux pattern: FP64 all-pairs pass on the device
    HIPCHECK(launch_psi(s, const_cast<double *>(s.psi), st));
    if ((rc = reset_state(h))) return rc;
    HIPCHECK(hipStreamSynchronize(st));  // host vectors above go out of scope
    h->pub2int.swap(pub2int);
    *out = guard.release();
    return COIL_OK;
}

extern "C" int coil_step(coil_t *h) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    return enqueue_step(h);
}

extern "C" int coil_compute_field(coil_t *h) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    HIPCHECK(launch_field_any(h, h->ds, h->stream));
    HIPCHECK(launch_field_finalize(h->ds, h->rc, h->stream));
    return COIL_OK;
}

static int read_scalars(coil_t *h, Scalars *out) {
    HIPCHECK(hipMemcpyAsync(out, h->ds.sc, sizeof(Scalars), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    return COIL_OK;
}

static int max_B(coil_t *h, double *out) {
    const int N = h->ds.N;
    std::vector<double> br(N), bz(N);
    HIPCHECK(hipMemcpyAsync(br.data(), h->ds.Br, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipMemcpyAsync(bz.data(), h->ds.Bz, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    double m = 0.0;
    for (int i = 0; i < N; ++i) m = std::max(m, std::hypot(br[i], bz[i]));
    *out = m;
    return COIL_OK;
}

static int run_steps(coil_t *h, int64_t nsteps, int64_t report_every, coil_report_fn cb, void *user);

extern "C" int coil_run(coil_t *h, int64_t nsteps, int64_t report_every, coil_report_fn cb, void *user) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (nsteps < 0 || report_every < 0) return fail(COIL_E_INVAL, "negative step count");
    const int rc = run_steps(h, nsteps, report_every, cb, user);
    if (h->side_pending) (void)join_side(h);  // an error path left side-stream work unjoined
    return rc;
}

static int run_steps(coil_t *h, int64_t nsteps, int64_t report_every, coil_report_fn cb, void *user) {
    int rc;
    int64_t done = 0;
    while (done < nsteps) {
        int64_t chunk = nsteps - done;
        if (report_every > 0 && cb) chunk = std::min<int64_t>(chunk, report_every);
        int64_t k = 0;
        if (h->gexec && !h->timing && h->gsteps > 0) {
            if ((rc = join_side(h))) return rc;
            for (; k + h->gsteps <= chunk; k += h->gsteps) HIPCHECK(hipGraphLaunch(h->gexec, h->stream));
        }
        for (; k < chunk; ++k)
            if ((rc = enqueue_step(h, true))) return rc;
        if ((rc = join_side(h))) return rc;
        done += chunk;
        if (report_every > 0 && cb) {
            Scalars sc;
            if ((rc = read_scalars(h, &sc))) return rc;
            double mb = 0.0;
            if ((rc = max_B(h, &mb))) return rc;
            const double t = (double)sc.step * h->rc.dt;
            const double It0 = h->plan.coils[0].I0e * h->plan.coils[0].ne2 + h->plan.coils[0].dIt / h->rc.dt * t;
            const double diag[8] = {t, (double)sc.step, It0, mb, sc.Tpeak, sc.Q, sc.sumU, sc.maxx};
            cb(diag, 8, user);
            if (sc.status) return fail(COIL_E_NONFINITE, "non-finite state (status 0x%x) at step %lld", sc.status, sc.step);
        }
    }
    Scalars sc;
    if ((rc = read_scalars(h, &sc))) return rc;
    if (sc.status) return fail(COIL_E_NONFINITE, "non-finite state (status 0x%x) at step %lld", sc.status, sc.step);
    return COIL_OK;
}

static int field_len(coil_t *h, int field, int *len, int *per_wire) {
    *per_wire = 0;
    switch (field) {
        case COIL_F_QW:
        case COIL_F_UW:
        case COIL_F_ONSET: case COIL_F_QUENCH: case COIL_F_Q_ONSET: case COIL_F_Q_QUENCH:
        case COIL_F_T_QUENCH: case COIL_F_P_QUENCH:
            *per_wire = 1;
            *len = h->ds.Nw;
            return COIL_OK;
        case COIL_F_I: case COIL_F_J: case COIL_F_BR: case COIL_F_BZ: case COIL_F_T: case COIL_F_PHI:
        case COIL_F_E: case COIL_F_EP: case COIL_F_U: case COIL_F_Q: case COIL_F_PSI: case COIL_F_R:
        case COIL_F_Z: case COIL_F_DI: case COIL_F_JC:
            *len = h->ds.N;
            return COIL_OK;
        case COIL_F_IH:
            if (!h->ds.IH) return fail(COIL_E_INVAL, "COIL_F_IH needs the subelement model (subelements > 0)");
            *len = h->ds.N;
            return COIL_OK;
        case COIL_F_EM_SUBSTEPS:
            if (!h->ds.emsub) return fail(COIL_E_INVAL, "COIL_F_EM_SUBSTEPS needs the variable step (em_tol > 0)");
            *per_wire = 1;
            *len = h->ds.Nw;
            return COIL_OK;
        default:
            return fail(COIL_E_INVAL, "unknown field %d", field);
    }
}

extern "C" int coil_get(coil_t *h, int32_t field, double *dst, int64_t count, int32_t dst_on_device) {
    if (!h || !dst) return fail(COIL_E_INVAL, "NULL argument");
    int len, pw, rc;
    if ((rc = field_len(h, field, &len, &pw))) return rc;
    if (count < len) return fail(COIL_E_INVAL, "count %lld < field length %d", (long long)count, len);
    const DevState &s = h->ds;
    hipStream_t st = h->stream;
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (field == COIL_F_R || field == COIL_F_Z) {
        const std::vector<double> &v = field == COIL_F_R ? h->r_pub : h->z_pub;
        HIPCHECK(hipMemcpyAsync(dst, v.data(), sizeof(double) * len,
                                dst_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        return COIL_OK;
    }
    if (pw) {
        const double *src = nullptr;
        switch (field) {
            case COIL_F_QW: src = s.Qw; break;
            case COIL_F_UW: src = s.Uw; break;
            case COIL_F_ONSET: src = s.onset; break;
            case COIL_F_QUENCH: src = s.quench; break;
            case COIL_F_Q_ONSET: src = s.Qon; break;
            case COIL_F_Q_QUENCH: src = s.Qqu; break;
            case COIL_F_T_QUENCH: src = s.Tqu; break;
            case COIL_F_EM_SUBSTEPS: src = s.emsub; break;
            default: src = s.Pqu; break;
        }
        HIPCHECK(hipMemcpyAsync(dst, src, sizeof(double) * len, kind, st));
        if (!dst_on_device) HIPCHECK(hipStreamSynchronize(st));
        return COIL_OK;
    }
    const double *src = nullptr;
    switch (field) {
        case COIL_F_I: src = s.I; break;
        case COIL_F_BR: src = s.Br; break;
        case COIL_F_BZ: src = s.Bz; break;
        case COIL_F_T: src = s.T[0]; break;
        case COIL_F_PHI: src = s.Phi; break;
        case COIL_F_E: src = s.E; break;
        case COIL_F_EP: src = s.Ep; break;
        case COIL_F_U: src = s.u[0]; break;
        case COIL_F_Q: src = s.q; break;
        case COIL_F_PSI: src = s.psi; break;
        case COIL_F_DI: src = s.dI; break;
        case COIL_F_JC: src = s.Jc; break;
        case COIL_F_J: src = s.I; break;
        case COIL_F_IH: src = s.IH; break;
        default: return fail(COIL_E_INVAL, "field %d not readable", field);
    }
    double *stage = dst_on_device ? dst : s.tmp;
    HIPCHECK(launch_gather(src, s.perm, len, stage, st));
    if (!dst_on_device) {
        HIPCHECK(hipMemcpyAsync(dst, s.tmp, sizeof(double) * len, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
    }
    if (field == COIL_F_J) {
        // J = I / d^2 per coil (public order is coil-concatenated)
        if (dst_on_device) {
            std::vector<double> tmp(len);
            HIPCHECK(hipMemcpyAsync(tmp.data(), dst, sizeof(double) * len, hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            for (const CoilDev &d : h->plan.coils)
                for (int i = d.off; i < d.off + d.n; ++i) tmp[i] /= d.d * d.d;
            HIPCHECK(hipMemcpyAsync(dst, tmp.data(), sizeof(double) * len, hipMemcpyHostToDevice, st));
            HIPCHECK(hipStreamSynchronize(st));
        } else {
            for (const CoilDev &d : h->plan.coils)
                for (int i = d.off; i < d.off + d.n; ++i) dst[i] /= d.d * d.d;
        }
    }
    return COIL_OK;
}

extern "C" int coil_set_state(coil_t *h, int32_t field, const double *src, int64_t count,
                              int32_t src_on_device) {
    if (!h || !src) return fail(COIL_E_INVAL, "NULL argument");
    if (field != COIL_F_I && field != COIL_F_T) return fail(COIL_E_INVAL, "field %d is not settable", field);
    const DevState &s = h->ds;
    if (count < s.N) return fail(COIL_E_INVAL, "count %lld < %d", (long long)count, s.N);
    hipStream_t st = h->stream;
    const double *pub = src;
    if (!src_on_device) {
        HIPCHECK(hipMemcpyAsync(s.tmp, src, sizeof(double) * s.N, hipMemcpyHostToDevice, st));
        pub = s.tmp;
    }
    if (field == COIL_F_I) {
        HIPCHECK(launch_scatter(pub, s.perm, s.N, s.I, st));
    } else {
        HIPCHECK(launch_scatter(pub, s.perm, s.N, s.T[0], st));
        HIPCHECK(launch_u_of_T(s, h->rc, st));
    }
    HIPCHECK(hipStreamSynchronize(st));
    return COIL_OK;
}

extern "C" int coil_scalars(coil_t *h, double *dst, int32_t n) {
    if (!h || !dst) return fail(COIL_E_INVAL, "NULL argument");
    Scalars sc;
    int rc;
    if ((rc = read_scalars(h, &sc))) return rc;
    double *misc = at<double>(h, h->plan.misc_b);
    HIPCHECK(launch_stored(h->ds, misc, h->stream));
    double stored = 0.0;
    HIPCHECK(hipMemcpyAsync(&stored, misc, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    CgScalars cg{};
    if (h->ds.cg) {
        HIPCHECK(hipMemcpyAsync(&cg, h->ds.cg, sizeof(cg), hipMemcpyDeviceToHost, h->stream));
        HIPCHECK(hipStreamSynchronize(h->stream));
    }
    const double res = cg.rho0 > 0.0 ? std::sqrt(std::max(0.0, cg.rho) / cg.rho0) : 0.0;
    const double v[15] = {(double)sc.step * h->rc.dt, (double)sc.step, sc.Q, sc.Tpeak, sc.sumU, sc.maxx,
                          sc.Qout, stored, (double)sc.status, (double)sc.Tpeak_pub, (double)sc.Tpeak_step,
                          (double)h->ds.nsub, (double)h->ds.nitems, (double)cg.iters, res};
    for (int i = 0; i < n && i < 15; ++i) dst[i] = v[i];
    return COIL_OK;
}

extern "C" int coil_reset(coil_t *h) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    int rc = reset_state(h);
    if (rc) return rc;
    HIPCHECK(hipStreamSynchronize(h->stream));
    return COIL_OK;
}

extern "C" int coil_timing(coil_t *h, int32_t enable) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (h->capturing) return fail(COIL_E_STATE, "timing cannot change during graph capture");
    if (enable < 0 || enable > 2) return fail(COIL_E_INVAL, "enable must be 0, 1 or 2");
    int rc = t_flush(h);
    if (rc) return rc;
    h->timing = enable != 0;
    h->timing_all = enable == 1;
    if (h->timing)
        for (int i = 0; i < 4; ++i) {
            h->ms[i] = 0.0;
            h->launches[i] = 0;
        }
    return COIL_OK;
}

extern "C" int coil_timing_read(coil_t *h, double *ms, int64_t *launches, int32_t n) {
    if (!h || !ms || !launches) return fail(COIL_E_INVAL, "NULL argument");
    int rc = t_flush(h);
    if (rc) return rc;
    for (int i = 0; i < n && i < 4; ++i) {
        ms[i] = h->ms[i];
        launches[i] = h->launches[i];
    }
    return COIL_OK;
}

extern "C" int coil_graph(coil_t *h, int64_t steps) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (steps < 0) return fail(COIL_E_INVAL, "steps < 0");
    if (h->gexec) {
        HIPCHECK(hipGraphExecDestroy(h->gexec));
        h->gexec = nullptr;
    }
    if (h->graph) {
        HIPCHECK(hipGraphDestroy(h->graph));
        h->graph = nullptr;
    }
    h->gsteps = 0;
    if (steps == 0) return COIL_OK;
    if (h->stream == nullptr) return fail(COIL_E_STATE, "graph capture needs a non-default stream");
    if (h->timing) return fail(COIL_E_STATE, "disable timing before capturing a graph");
    h->capturing = true;
    HIPCHECK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = COIL_OK;
    for (int64_t k = 0; k < steps && rc == COIL_OK; ++k) rc = enqueue_step(h, true);
    if (rc == COIL_OK) rc = join_side(h);  // the side stream rejoins before the capture ends
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    h->capturing = false;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(COIL_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    h->graph = g;
    HIPCHECK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    h->gsteps = steps;
    return COIL_OK;
}

extern "C" void coil_destroy(coil_t *h) {
    if (!h) return;
    if (h->stream || h->ws) (void)hipStreamSynchronize(h->stream);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    for (auto &p : h->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    delete h;
}

extern "C" int coil_host_ellip(double m1, int32_t precision, double *K, double *E) {
    if (!K || !E) return fail(COIL_E_INVAL, "NULL argument");
    if (!(m1 > 0.0 && m1 <= 1.0)) return fail(COIL_E_INVAL, "m1 must be in (0, 1]");
    if (precision == COIL_FP64) {
        host_ellip_f64(m1, K, E);
    } else if (precision == COIL_MIXED) {
        float k, e;
        host_ellip_f32((float)m1, &k, &e);
        *K = k;
        *E = e;
    } else {
        return fail(COIL_E_INVAL, "unknown precision");
    }
    return COIL_OK;
}

// ------------------------------------------------------------------ parameters
extern "C" int coil_set_params(coil_t *h, const double *c_wire, const double *ramp) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (h->capturing) return fail(COIL_E_STATE, "cannot change parameters during graph capture");
    if (c_wire) {
        for (int w = 0; w < h->ds.Nw; ++w)
            if (!std::isfinite(c_wire[w])) return fail(COIL_E_INVAL, "non-finite c_wire at %d", w);
        HIPCHECK(hipMemcpyAsync((void *)h->ds.cw, c_wire, sizeof(double) * h->ds.Nw, hipMemcpyHostToDevice,
                                h->stream));
    }
    if (ramp) {
        for (size_t i = 0; i < h->plan.coils.size(); ++i) {
            if (!std::isfinite(ramp[i])) return fail(COIL_E_INVAL, "non-finite ramp of coil %zu", i);
            h->plan.coils[i].dIt = ramp[i] * h->rc.dt;
        }
        HIPCHECK(hipMemcpyAsync((void *)h->ds.coils, h->plan.coils.data(), sizeof(CoilDev) * h->plan.coils.size(),
                                hipMemcpyHostToDevice, h->stream));
    }
    HIPCHECK(hipStreamSynchronize(h->stream));
    return COIL_OK;
}

// ------------------------------------------------------------------ transposed field pass (test hook)
extern "C" int coil_field_transpose(coil_t *h, const double *bbar_r, const double *bbar_z, double *out,
                                    int32_t on_device) {
    if (!h || !bbar_r || !bbar_z || !out) return fail(COIL_E_INVAL, "NULL argument");
    if (h->capturing) return fail(COIL_E_STATE, "not during graph capture");
    const DevState &s = h->ds;
    hipStream_t st = h->stream;
    const int N = s.N;
    // public inputs -> internal order in the Br / Bz buffers, then weights in place
    const double *pr = bbar_r, *pz = bbar_z;
    if (!on_device) {
        HIPCHECK(hipMemcpyAsync(s.tmp, bbar_r, sizeof(double) * N, hipMemcpyHostToDevice, st));
        HIPCHECK(launch_scatter(s.tmp, s.perm, N, s.Br, st));
        HIPCHECK(hipMemcpyAsync(s.tmp, bbar_z, sizeof(double) * N, hipMemcpyHostToDevice, st));
        HIPCHECK(launch_scatter(s.tmp, s.perm, N, s.Bz, st));
    } else {
        HIPCHECK(launch_scatter(pr, s.perm, N, s.Br, st));
        HIPCHECK(launch_scatter(pz, s.perm, N, s.Bz, st));
    }
    HIPCHECK(launch_field_weights(s, s.Br, s.Bz, st));
    double *partT = reinterpret_cast<double *>(s.part);
    // staging for public-order weights: the second half of the partial buffer
    // (partT needs at most nslot N doubles of its 2 nslot N)
    const int nsl = std::max({h->plan.nchunk_max, h->plan.nchunk_cap, h->plan.nslot_tz_max});
    double *wpub = partT + (size_t)nsl * N;  // nsl N + 2 N <= 2 part_slots N doubles
    if ((size_t)nsl * N + 2 * (size_t)N > 2 * (size_t)h->plan.part_slots * N)
        return fail(COIL_E_NOMEM, "partial buffer too small for the transposed pass");
    HIPCHECK(launch_fieldT_any(h, s.Br, s.Bz, wpub, partT, st));
    HIPCHECK(launch_fieldT_sum(s, partT, s.dI, 0, st));
    if (on_device) {
        HIPCHECK(launch_gather(s.dI, s.perm, N, out, st));
    } else {
        HIPCHECK(launch_gather(s.dI, s.perm, N, s.tmp, st));
        HIPCHECK(hipMemcpyAsync(out, s.tmp, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    }
    HIPCHECK(hipStreamSynchronize(st));
    return COIL_OK;
}

// ------------------------------------------------------------------ adjoint
namespace {
struct AdjLayout {
    size_t ckI, ckU, ckT, hBr, hBz, sI, sdI, sT, sBr, sBz, Ib, ub0, ub1, qb, wr, wz, partT, wpub, cb, dIb, total;
    long long nseg;
};

AdjLayout adj_layout(const Plan &p, long long K, long long C, int store_field) {
    AdjLayout L{};
    const size_t N = p.N, Nw = p.Nw, d8 = sizeof(double);
    L.nseg = (K + C - 1) / C;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        cur = (cur + 255) & ~size_t(255);
        const size_t o = cur;
        cur += bytes;
        return o;
    };
    L.ckI = take(d8 * N * L.nseg);
    L.ckU = take(d8 * N * L.nseg);
    L.ckT = take(d8 * N * L.nseg);
    if (store_field) {
        L.hBr = take(d8 * N * K);
        L.hBz = take(d8 * N * K);
    } else {
        L.sBr = take(d8 * N * C);
        L.sBz = take(d8 * N * C);
    }
    L.sI = take(d8 * N * C);
    L.sdI = take(d8 * N * C);
    L.sT = take(d8 * N * C * p.nsub);
    L.Ib = take(d8 * N);
    L.ub0 = take(d8 * N);
    L.ub1 = take(d8 * N);
    L.qb = take(d8 * N);
    L.wr = take(d8 * N);
    L.wz = take(d8 * N);
    L.partT = take(d8 * N * std::max({p.nchunk_max, p.nchunk_cap, p.nslot_tz_max}));
    L.wpub = take(d8 * N * 2);
    L.cb = take(d8 * Nw);
    L.dIb = take(d8 * Nw);
    L.total = (cur + 255) & ~size_t(255);
    return L;
}
}  // namespace

extern "C" int coil_adjoint_query(coil_t *h, int64_t nsteps, int32_t ckpt_every, int32_t store_field,
                                  size_t *bytes) {
    if (!h || !bytes) return fail(COIL_E_INVAL, "NULL argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(COIL_E_INVAL, "nsteps and ckpt_every must be >= 1");
    *bytes = adj_layout(h->plan, nsteps, ckpt_every, store_field != 0).total;
    return COIL_OK;
}

extern "C" int coil_adjoint(coil_t *h, int64_t nsteps, double wQ, double wTpeak, int32_t ckpt_every,
                            int32_t store_field, void *workspace, size_t bytes, double *g_c_wire,
                            double *g_ramp, double *objectives) {
    if (!h || !workspace || !g_c_wire || !g_ramp || !objectives) return fail(COIL_E_INVAL, "NULL argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(COIL_E_INVAL, "nsteps and ckpt_every must be >= 1");
    if (!std::isfinite(wQ) || !std::isfinite(wTpeak)) return fail(COIL_E_INVAL, "non-finite objective weight");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(COIL_E_INVAL, "workspace must be 256-byte aligned");
    if (h->capturing) return fail(COIL_E_STATE, "not during graph capture");
    if (h->ds.cg_defer) return fail(COIL_E_INVAL, "the adjoint covers the transport-only coupling (COIL_COUPLE_TRANSPORT)");
    if (h->ds.nsubel) return fail(COIL_E_INVAL, "the adjoint covers the wire model (subelements = 0)");
    if (h->ds.emsub) return fail(COIL_E_INVAL, "the adjoint covers the fixed step (em_tol = 0)");
    if (h->rc.adi) return fail(COIL_E_INVAL, "the adjoint covers the explicit heat step (COIL_HEAT_EXPLICIT)");
    const long long K = nsteps, C = ckpt_every;
    const int sf = store_field != 0;
    const AdjLayout L = adj_layout(h->plan, K, C, sf);
    if (bytes < L.total) return fail(COIL_E_NOMEM, "adjoint workspace of %zu bytes < %zu needed", bytes, L.total);
    char *wb = static_cast<char *>(workspace);
    auto P = [&](size_t off) { return reinterpret_cast<double *>(wb + off); };
    const DevState base = h->ds;
    const RunConst &rc = h->rc;
    hipStream_t st = h->stream;
    const int N = base.N, Nw = base.Nw, nsub = base.nsub;
    const size_t Ns = (size_t)N;
    int rc_ = COIL_OK;
    const bool timing = h->timing;
    h->timing = false;

    auto step_with = [&](const DevState &d, bool field) -> int {
        if (field) HIPCHECK(launch_field_any(h, d, st));
        HIPCHECK(launch_wire(d, rc, st));
        HIPCHECK(launch_heat_step(d, rc, st));
        HIPCHECK(launch_finalize(d, rc, st));
        return COIL_OK;
    };

    // forward pass with checkpoints (and the field history)
    if ((rc_ = reset_state(h))) return rc_;
    for (long long k = 0; k < K; ++k) {
        if (k % C == 0) {
            const long long sg = k / C;
            HIPCHECK(launch_copy(base.I, P(L.ckI) + sg * Ns, N, st));
            HIPCHECK(launch_copy(base.u[0], P(L.ckU) + sg * Ns, N, st));
            HIPCHECK(launch_copy(base.T[0], P(L.ckT) + sg * Ns, N, st));
        }
        DevState d = base;
        if (sf) {
            d.rec_Br = P(L.hBr) + k * Ns;
            d.rec_Bz = P(L.hBz) + k * Ns;
        }
        if ((rc_ = step_with(d, true))) return rc_;
    }
    Scalars sc;
    if ((rc_ = read_scalars(h, &sc))) return rc_;
    if (sc.status) {
        h->timing = timing;
        return fail(COIL_E_NONFINITE, "non-finite state in the forward pass (status 0x%x)", sc.status);
    }
    objectives[0] = sc.Q;
    objectives[1] = sc.Tpeak;
    const int e_star = sc.Tpeak_pub >= 0 ? h->pub2int[sc.Tpeak_pub] : -1;
    const double Cpk = rc.C0 * std::pow(sc.Tpeak / rc.T_ref, rc.cp_exp);

    // reverse sweep
    double *Ib = P(L.Ib), *ub = P(L.ub0), *ubn = P(L.ub1), *qb = P(L.qb);
    HIPCHECK(launch_fill(Ib, 0.0, N, st));
    HIPCHECK(launch_fill(ub, 0.0, N, st));
    HIPCHECK(launch_fill(P(L.cb), 0.0, Nw, st));
    HIPCHECK(launch_fill(P(L.dIb), 0.0, Nw, st));
    for (long long sg = L.nseg - 1; sg >= 0; --sg) {
        const long long k0 = sg * C, k1 = std::min(K, k0 + C);
        HIPCHECK(launch_copy(P(L.ckI) + sg * Ns, base.I, N, st));
        HIPCHECK(launch_copy(P(L.ckU) + sg * Ns, base.u[0], N, st));
        HIPCHECK(launch_copy(P(L.ckT) + sg * Ns, base.T[0], N, st));
        HIPCHECK(launch_set_step(base.sc, k0, st));
        for (long long k = k0; k < k1; ++k) {
            const long long j = k - k0;
            DevState d = base;
            d.rec_I = P(L.sI) + j * Ns;
            d.rec_dI = P(L.sdI) + j * Ns;
            d.rec_T = P(L.sT) + j * nsub * Ns;
            if (sf) {
                d.src_Br = P(L.hBr) + k * Ns;
                d.src_Bz = P(L.hBz) + k * Ns;
            } else {
                d.rec_Br = P(L.sBr) + j * Ns;
                d.rec_Bz = P(L.sBz) + j * Ns;
            }
            if ((rc_ = step_with(d, !sf))) return rc_;
        }
        for (long long k = k1 - 1; k >= k0; --k) {
            const long long j = k - k0;
            if (wTpeak != 0.0 && e_star >= 0 && k + 1 == sc.Tpeak_step)
                HIPCHECK(launch_add_at(ub, e_star, wTpeak / Cpk, st));
            HIPCHECK(launch_qbar_init(base, qb, wQ * rc.dt, st));
            for (int sub = nsub - 1; sub >= 0; --sub) {
                HIPCHECK(launch_heat_adj(base, rc, ub, ubn, P(L.sT) + (j * nsub + sub) * Ns, qb, st));
                std::swap(ub, ubn);
            }
            AdjPtrs a;
            a.I = P(L.sI) + j * Ns;
            a.T = P(L.sT) + j * nsub * Ns;
            a.Br = sf ? P(L.hBr) + k * Ns : P(L.sBr) + j * Ns;
            a.Bz = sf ? P(L.hBz) + k * Ns : P(L.sBz) + j * Ns;
            a.dI = P(L.sdI) + j * Ns;
            a.qbar = qb;
            a.Ibar = Ib;
            a.ubar = ub;
            a.wr = P(L.wr);
            a.wz = P(L.wz);
            a.cbar = P(L.cb);
            a.dItbar = P(L.dIb);
            HIPCHECK(launch_wire_adj(base, rc, a, st));
            HIPCHECK(launch_fieldT_any(h, a.wr, a.wz, P(L.wpub), P(L.partT), st));
            HIPCHECK(launch_fieldT_sum(base, P(L.partT), Ib, 1, st));
        }
    }
    std::vector<double> dIb(Nw);
    HIPCHECK(hipMemcpyAsync(g_c_wire, P(L.cb), sizeof(double) * Nw, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(dIb.data(), P(L.dIb), sizeof(double) * Nw, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    for (size_t ci = 0; ci < h->plan.coils.size(); ++ci) {
        const CoilDev &c = h->plan.coils[ci];
        double sgr = 0.0;
        for (int w = c.wire_off; w < c.wire_off + c.layers * c.turns; ++w) sgr += dIb[w];
        g_ramp[ci] = rc.dt * sgr;
    }
    if ((rc_ = reset_state(h))) return rc_;
    HIPCHECK(hipStreamSynchronize(st));
    h->timing = timing;
    return COIL_OK;
}

// ------------------------------------------------------------------ autotuner
namespace {
std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int apply_tz(coil_t *h, int nsplit) {
    Plan q = h->plan;
    build_tz(q, nsplit, h->tz_force_w);
    if (q.tz_items.size() > h->plan.tz_cap || q.nslot_tz_max > h->plan.part_slots)
        return fail(COIL_E_INVAL, "translation split %d exceeds the planned capacity", nsplit);
    HIPCHECK(hipMemcpyAsync((void *)h->tz.items, q.tz_items.data(), sizeof(TzItem) * q.tz_items.size(),
                            hipMemcpyHostToDevice, h->stream));
    for (size_t i = 0; i < q.coils.size(); ++i) h->plan.coils[i].nslot_tz = q.coils[i].nslot_tz;
    HIPCHECK(hipMemcpyAsync((void *)h->ds.coils, h->plan.coils.data(), sizeof(CoilDev) * h->plan.coils.size(),
                            hipMemcpyHostToDevice, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    const size_t cap = h->plan.tz_cap;
    h->plan.tz_items = q.tz_items;
    h->plan.tz_cap = cap;
    h->plan.nslot_tz_max = q.nslot_tz_max;
    h->plan.tz_evals = q.tz_evals;
    h->tz.n = (int)q.tz_items.size();
    h->tz_split = nsplit;
    return COIL_OK;
}

std::string tune_key(const coil_t *h) {
    long double pairs = 0;
    for (const CoilDev &d : h->plan.coils) pairs += (long double)d.n * (d.n - 1);
    const int lg = pairs > 1 ? (int)std::floor(std::log2((double)pairs)) : 0;
    char buf[128];
    snprintf(buf, sizeof(buf), "%s/%s/p%d/c%zu", arch_name().c_str(), h->rc.prec == COIL_MIXED ? "mixed" : "fp64",
             lg, h->plan.coils.size());
    return buf;
}

int apply_tiles(coil_t *h, int tb, int nch, int grid) {
    Plan q = h->plan;
    build_items(q, tb, nch, 0);
    if (q.items.size() > h->plan.items_cap && q.items.size() > h->plan.items.size())
        return fail(COIL_E_INVAL, "tile shape needs %zu work items, capacity %zu", q.items.size(), h->plan.items_cap);
    if (q.nchunk_max > std::max(h->plan.nchunk_cap, h->plan.nchunk_max))
        return fail(COIL_E_INVAL, "tile shape needs %d source chunks", q.nchunk_max);
    HIPCHECK(hipMemcpyAsync((void *)h->ds.items, q.items.data(), sizeof(PairItem) * q.items.size(),
                            hipMemcpyHostToDevice, h->stream));
    HIPCHECK(hipMemcpyAsync((void *)h->ds.coils, q.coils.data(), sizeof(CoilDev) * q.coils.size(),
                            hipMemcpyHostToDevice, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    const size_t cap = h->plan.items_cap;
    const int pcap = h->plan.nchunk_cap;
    h->plan.items = q.items;
    h->plan.coils = q.coils;
    h->plan.tile_targets = q.tile_targets;
    h->plan.nchunk_max = q.nchunk_max;
    h->plan.items_cap = cap;
    h->plan.nchunk_cap = pcap;
    h->ds.nitems = (int)q.items.size();
    h->ds.tile_targets = tb;
    h->grid_limit = grid;
    return COIL_OK;
}
}  // namespace

extern "C" int coil_set_widths(coil_t *h, int32_t w) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (!(w == 0 || (w >= 2 && w <= 8))) return fail(COIL_E_INVAL, "w must be 0 or in [2, 8]");
    if (h->capturing) return fail(COIL_E_STATE, "not during graph capture");
    int rc = coil_graph(h, 0);
    if (rc) return rc;
    h->tz_force_w = w;
    return apply_tz(h, h->tz_split);
}

extern "C" int coil_set_tiles(coil_t *h, int32_t tile_targets, int32_t chunks, int32_t grid_limit) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (!(tile_targets == 64 || tile_targets == 128 || tile_targets == 256))
        return fail(COIL_E_INVAL, "tile_targets must be 64, 128 or 256");
    if (chunks < 0 || chunks > kMaxChunks) return fail(COIL_E_INVAL, "chunks must be in [0, %d]", kMaxChunks);
    if (grid_limit < 0) return fail(COIL_E_INVAL, "grid_limit must be >= 0");
    if (h->capturing) return fail(COIL_E_STATE, "not during graph capture");
    int rc = coil_graph(h, 0);
    if (rc) return rc;
    h->ds.algo_tz = 0;
    h->ds.algo_fft = 0;
    h->plan.algo = COIL_ALGO_DIRECT;
    return apply_tiles(h, tile_targets, chunks, grid_limit);
}

extern "C" int coil_autotune(coil_t *h, int32_t reps, const char *cache_path, int32_t *chosen) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (reps < 1) return fail(COIL_E_INVAL, "reps must be >= 1");
    if (h->capturing) return fail(COIL_E_STATE, "not during graph capture");
    int rc = coil_graph(h, 0);
    if (rc) return rc;
    const std::string key = tune_key(h);
    // choice: algo (1 direct, 2 translation), then (tile_targets, chunks, grid) or (split)
    auto apply = [&](int algo, int a, int b, int c) -> int {
        h->ds.algo_fft = 0;
        if (algo == COIL_ALGO_FFT) {  // only where its spectra were made at init
            if (!h->plan.fft) return fail(COIL_E_INVAL, "the fast-convolution pass was not set up");
            h->ds.algo_tz = 0;
            h->ds.algo_fft = 1;
            h->plan.algo = COIL_ALGO_FFT;
            h->grid_limit = 0;
            return COIL_OK;
        }
        if (algo == COIL_ALGO_TRANSLATION) {
            h->ds.algo_tz = 1;
            h->plan.algo = COIL_ALGO_TRANSLATION;
            h->grid_limit = 0;  // the work-queue launch (a DIRECT candidate may have set a grid)
            return apply_tz(h, a);
        }
        h->ds.algo_tz = 0;
        h->plan.algo = COIL_ALGO_DIRECT;
        return apply_tiles(h, a, b, c);
    };
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[512];
            int ba = 0, b1 = 0, b2 = 0, b3 = 0;
            while (fgets(line, sizeof(line), f)) {
                char k[200];
                int al, x1, x2, x3;
                double ms;
                if (sscanf(line, "{\"key\": \"%199[^\"]\", \"algo\": %d, \"p1\": %d, \"p2\": %d, \"p3\": %d, \"ms\": %lf}",
                           k, &al, &x1, &x2, &x3, &ms) == 6 && key == k) {
                    ba = al; b1 = x1; b2 = x2; b3 = x3;
                }
            }
            fclose(f);
            if (ba) {
                if ((rc = apply(ba, b1, b2, b3))) return rc;
                if (chosen) { chosen[0] = ba; chosen[1] = b1; chosen[2] = b2; chosen[3] = b3; }
                return COIL_OK;
            }
        }
    }
    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        cus = prop.multiProcessorCount;
    hipEvent_t ea = nullptr, eb = nullptr;
    struct EvGuard {  // the events are released on every return path
        hipEvent_t *a, *b;
        ~EvGuard() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } guard{&ea, &eb};
    HIPCHECK(hipEventCreate(&ea));
    HIPCHECK(hipEventCreate(&eb));
    double best = INFINITY;
    int ba = h->plan.algo, b1 = 0, b2 = 0, b3 = 0;
    struct Cand { int algo, a, b, c; };
    std::vector<Cand> cands;
    if (h->plan.fft) cands.push_back({COIL_ALGO_FFT, 0, 0, 0});
    for (int sp : {4, 8, 16, 32, 64}) cands.push_back({COIL_ALGO_TRANSLATION, sp, 0, 0});
    for (int tb : {64, 128, 256})
        for (int ch : {1, 2, 4, 8, kMaxChunks})
            for (int g : {0, 2 * cus, 4 * cus}) cands.push_back({COIL_ALGO_DIRECT, tb, ch, g});
    // Every candidate's first launch is timed as a screen: only candidates within
    // 3x of the best so far get the `reps` timed launches, and a family (algorithm)
    // whose first three candidates all stay beyond 3x is not tried further.
    int fam_tried[4] = {0, 0, 0, 0};
    double fam_best[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    auto elapsed = [&](float *ms) -> int {
        HIPCHECK(hipEventRecord(eb, h->stream));
        HIPCHECK(hipEventSynchronize(eb));
        HIPCHECK(hipEventElapsedTime(ms, ea, eb));
        return COIL_OK;
    };
    for (const Cand &cd : cands) {
        if (fam_tried[cd.algo] >= 3 && fam_best[cd.algo] > 3.0 * best) continue;
        if (apply(cd.algo, cd.a, cd.b, cd.c)) continue;  // over capacity: skip
        float ms = 0.f;
        HIPCHECK(hipEventRecord(ea, h->stream));
        HIPCHECK(launch_field_any(h, h->ds, h->stream));
        if ((rc = elapsed(&ms))) return rc;
        ++fam_tried[cd.algo];
        fam_best[cd.algo] = std::min(fam_best[cd.algo], (double)ms);
        if (ms > 3.0 * best) continue;
        HIPCHECK(hipEventRecord(ea, h->stream));
        for (int r = 0; r < reps; ++r) HIPCHECK(launch_field_any(h, h->ds, h->stream));
        if ((rc = elapsed(&ms))) return rc;
        fam_best[cd.algo] = std::min(fam_best[cd.algo], (double)ms / reps);
        if (ms / reps < best) {
            best = ms / reps;
            ba = cd.algo; b1 = cd.a; b2 = cd.b; b3 = cd.c;
        }
    }
    g_err.clear();
    if ((rc = apply(ba, b1, b2, b3))) return rc;
    if (chosen) { chosen[0] = ba; chosen[1] = b1; chosen[2] = b2; chosen[3] = b3; }
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"key\": \"%s\", \"algo\": %d, \"p1\": %d, \"p2\": %d, \"p3\": %d, \"ms\": %.6f}\n",
                    key.c_str(), ba, b1, b2, b3, best);
            fclose(f);
        }
    }
    return COIL_OK;
}

extern "C" int coil_field_stats(coil_t *h, double *out, int32_t n) {
    if (!h || !out) return fail(COIL_E_INVAL, "NULL argument");
    double pairs = 0.0;
    for (const CoilDev &d : h->plan.coils) pairs += (double)d.n * (double)(d.n - 1);
    const bool tz = h->ds.algo_tz != 0, ff = h->ds.algo_fft != 0;
    const int nit = ff ? h->plan.fftp.nbins : tz ? (int)h->plan.tz_items.size() : (int)h->plan.items.size();
    const int resident = h->rc.prec == COIL_MIXED ? h->tz.grid32 : h->tz.grid64;
    const int wg = ff ? nit
                   : h->grid_limit > 0 ? std::min(h->grid_limit, nit)
                   : tz && resident > 0 ? std::min(resident, nit)
                                        : nit;
    const double v[6] = {pairs, ff ? 0.0 : tz ? h->plan.tz_evals : pairs, ff ? 3.0 : tz ? 2.0 : 1.0, (double)nit,
                         (double)h->ds.tile_targets, (double)wg};
    for (int i = 0; i < n && i < 6; ++i) out[i] = v[i];
    return COIL_OK;
}

// ------------------------------------------------------------------ probes
extern "C" int coil_field_at(coil_t *h, int64_t npts, const double *r, const double *z, double *Br, double *Bz) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (npts < 0) return fail(COIL_E_INVAL, "npts < 0");
    if (npts == 0) return COIL_OK;
    if (!r || !z || !Br || !Bz) return fail(COIL_E_INVAL, "NULL argument");
    for (int64_t i = 0; i < npts; ++i)
        if (!std::isfinite(r[i]) || !std::isfinite(z[i]) || r[i] < 0.0)
            return fail(COIL_E_INVAL, "probe %lld: r must be finite and >= 0, z finite", (long long)i);
    const DevState &s = h->ds;
    hipStream_t st = h->stream;
    // staging: the partial buffer holds >= 4 N doubles; probes go in chunks of N
    double *buf = reinterpret_cast<double *>(s.part);
    const int64_t chunk = std::max<int64_t>(1, s.N);
    for (int64_t p0 = 0; p0 < npts; p0 += chunk) {
        const int np = (int)std::min<int64_t>(chunk, npts - p0);
        double *dr = buf, *dz = buf + chunk, *ob = buf + 2 * chunk, *oz = buf + 3 * chunk;
        HIPCHECK(hipMemcpyAsync(dr, r + p0, sizeof(double) * np, hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(dz, z + p0, sizeof(double) * np, hipMemcpyHostToDevice, st));
        HIPCHECK(launch_probe(s, at<double>(h, h->plan.zphys_b), np, dr, dz, ob, oz, st));
        HIPCHECK(hipMemcpyAsync(Br + p0, ob, sizeof(double) * np, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipMemcpyAsync(Bz + p0, oz, sizeof(double) * np, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
    }
    return COIL_OK;
}

// ------------------------------------------------------------------ probes without allocation
// Scratch of coil_field_at_noalloc: the probes' per-chunk partial sums.  Each
// GPU the library runs on holds its own copy until the process ends; host
// code uses only the device address found by hipGetSymbolAddress (kept per
// device), never the array's name.
static __device__ __align__(256) double2 scratch[COIL_FIELD_AT_SCRATCH_BYTES / sizeof(double2)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2 *g_scratch_ptr[kMaxDevices] = {};

// the current device's scratch address (looked up once per device)
int scratch_for_current_device(double2 **out) {
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(COIL_E_HIP, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(COIL_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double2 *>(p);
    }
    *out = g_scratch_ptr[dev];
    return COIL_OK;
}
}  // namespace

extern "C" int coil_field_at_noalloc(coil_t *h, int64_t npts, const double *r, const double *z, double *Br,
                                     double *Bz) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    if (npts < 0) return fail(COIL_E_INVAL, "npts < 0");
    const int64_t cap = (int64_t)(COIL_FIELD_AT_SCRATCH_BYTES / sizeof(double2));
    if (npts > cap) return fail(COIL_E_INVAL, "npts %lld exceeds the %lld probes the static scratch holds",
                                (long long)npts, (long long)cap);
    if (npts == 0) return COIL_OK;
    if (!r || !z || !Br || !Bz) return fail(COIL_E_INVAL, "NULL argument");
    if (!h->scratch) return fail(COIL_E_STATE, "no scratch address for this handle's device");
    const DevState &s = h->ds;
    // source chunks: about 2048 workgroups in all, at most one chunk per LDS
    // stage of sources, and within the scratch
    const int np = (int)npts;
    const long long nb = (np + 255) / 256;
    long long nchunk = std::max<long long>(1, (2048 + nb - 1) / nb);
    nchunk = std::min<long long>(nchunk, std::max(1, (s.N + kStage - 1) / kStage));
    nchunk = std::max<long long>(1, std::min<long long>(nchunk, cap / np));
    HIPCHECK(launch_probe_chunked(s, at<double>(h, h->plan.zphys_b), np, r, z, Br, Bz, h->scratch, (int)nchunk,
                                  h->stream));
    return COIL_OK;
}

// ------------------------------------------------------------------ snapshots
namespace {
struct SnapHeader {
    char magic[8];
    int64_t N, Nw, step;
    double Q, Tpeak, Qout;
    int64_t Tpeak_pub, Tpeak_step;
    uint32_t status, nsub;
    uint32_t nsubel, pad;
};
// I, u, T, Phi, the per-wire Q_w and diagnostics, and I_H in the subelement model
size_t snap_bytes(const coil_t *h) {
    return sizeof(SnapHeader) +
           sizeof(double) * ((h->ds.IH ? 5 : 4) * (size_t)h->ds.N + 7 * (size_t)h->ds.Nw);
}
}  // namespace

extern "C" int coil_save(coil_t *h, void *host_buf, size_t bytes, size_t *needed) {
    if (!h) return fail(COIL_E_INVAL, "handle is NULL");
    const size_t need = snap_bytes(h);
    if (needed) *needed = need;
    if (!host_buf) return COIL_OK;
    if (bytes < need) return fail(COIL_E_INVAL, "snapshot buffer of %zu bytes < %zu", bytes, need);
    Scalars sc;
    int rc = read_scalars(h, &sc);
    if (rc) return rc;
    SnapHeader hd{};
    std::memcpy(hd.magic, "COILSNP3", 8);
    hd.N = h->ds.N;
    hd.Nw = h->ds.Nw;
    hd.step = sc.step;
    hd.Q = sc.Q;
    hd.Tpeak = sc.Tpeak;
    hd.Qout = sc.Qout;
    hd.Tpeak_pub = sc.Tpeak_pub;
    hd.Tpeak_step = sc.Tpeak_step;
    hd.status = sc.status;
    hd.nsub = (uint32_t)h->ds.nsub;
    hd.nsubel = (uint32_t)h->ds.nsubel;
    char *b = static_cast<char *>(host_buf);
    std::memcpy(b, &hd, sizeof(hd));
    double *d = reinterpret_cast<double *>(b + sizeof(hd));
    const size_t N = h->ds.N;
    hipStream_t st = h->stream;
    // internal order: a snapshot restores into a handle of the same configuration
    HIPCHECK(hipMemcpyAsync(d, h->ds.I, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(d + N, h->ds.u[0], sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(d + 2 * N, h->ds.T[0], sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(d + 3 * N, h->ds.Phi, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(d + 4 * N, h->ds.Qw, sizeof(double) * h->ds.Nw, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(d + 4 * N + h->ds.Nw, h->ds.onset, sizeof(double) * 6 * h->ds.Nw, hipMemcpyDeviceToHost,
                            st));
    if (h->ds.IH)
        HIPCHECK(hipMemcpyAsync(d + 4 * N + 7 * h->ds.Nw, h->ds.IH, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    return COIL_OK;
}

extern "C" int coil_load(coil_t *h, const void *host_buf, size_t bytes) {
    if (!h || !host_buf) return fail(COIL_E_INVAL, "NULL argument");
    if (h->capturing) return fail(COIL_E_STATE, "not during graph capture");
    if (bytes < sizeof(SnapHeader)) return fail(COIL_E_INVAL, "snapshot too small");
    SnapHeader hd;
    std::memcpy(&hd, host_buf, sizeof(hd));
    if (std::memcmp(hd.magic, "COILSNP3", 8) != 0) return fail(COIL_E_INVAL, "not a coil snapshot");
    if (hd.N != h->ds.N || hd.Nw != h->ds.Nw || (int)hd.nsub != h->ds.nsub || (int)hd.nsubel != h->ds.nsubel)
        return fail(COIL_E_INVAL, "snapshot of a different configuration");
    if (bytes < snap_bytes(h)) return fail(COIL_E_INVAL, "snapshot truncated");
    int rc = reset_state(h);  // clears scratch buffers and partial sums
    if (rc) return rc;
    const double *d = reinterpret_cast<const double *>(static_cast<const char *>(host_buf) + sizeof(hd));
    const size_t N = h->ds.N;
    hipStream_t st = h->stream;
    HIPCHECK(hipMemcpyAsync(h->ds.I, d, sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(h->ds.u[0], d + N, sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(h->ds.T[0], d + 2 * N, sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(h->ds.Phi, d + 3 * N, sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(h->ds.Qw, d + 4 * N, sizeof(double) * h->ds.Nw, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(h->ds.onset, d + 4 * N + h->ds.Nw, sizeof(double) * 6 * h->ds.Nw, hipMemcpyHostToDevice,
                            st));
    if (h->ds.IH)
        HIPCHECK(hipMemcpyAsync(h->ds.IH, d + 4 * N + 7 * h->ds.Nw, sizeof(double) * N, hipMemcpyHostToDevice, st));
    Scalars sc{};
    sc.Q = hd.Q;
    sc.Tpeak = hd.Tpeak;
    sc.Qout = hd.Qout;
    sc.step = hd.step;
    sc.Tpeak_pub = hd.Tpeak_pub;
    sc.Tpeak_step = hd.Tpeak_step;
    sc.status = hd.status;
    HIPCHECK(hipMemcpyAsync(h->ds.sc, &sc, sizeof(sc), hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    return COIL_OK;
}
