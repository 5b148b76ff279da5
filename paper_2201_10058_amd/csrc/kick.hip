// Changeover-weighted kick with fused close-encounter pair emission.
//
// Paper: GENGA II Sect. 2 (interaction part H_B of the democratic-heliocentric
// splitting, eq. Hb; critical radius eq. rcrit), Sect. 6.2 (the changeover acts
// on 0.1 < r/r_crit < 1 with the form of Chambers 1999 eq. 10), Appendix A
// (kick with the close-encounter pre-check), Appendix B (fixed pair-list order
// for exact reproducibility).
//
// Design for gfx950 (wave64, 256 CUs):
//  * The work is cut into tiles: a block of rows of one system against a
//    range of its columns.  A single system uses an implicit 2-D grid of tiles
//    (row blocks x column slices); a batch of systems uses a host-built,
//    cost-sorted tile list walked by a persistent grid.
//  * Each block stages NT columns (x, y, z, m, rc^2) in LDS; every lane
//    owns IPT rows and streams the tile with broadcast LDS reads.  Per
//    interaction the FP64 fast path is 3 sub, 3 mul/fma for r^2, v_rsq_f64
//    with a first-order correction folded into m r^-3 (5 ops), 3 fma
//    accumulations and one compare of r^2 against a wave-uniform bound (the
//    largest rc^2 among the wave's rows and the tile's columns, which is at
//    least max(rc_i^2, rc_j^2)).  Pairs under the bound take a divergent slow
//    path that makes the exact test r^2 < max(rc_i^2, rc_j^2), evaluates K
//    inside it, records encounter pairs and detects the self pair and
//    coincident bodies.
//  * Partial sums per column slice go to the workspace; k_kick_reduce adds
//    them in slice order (no atomics), applies v += h a and prepares the pair
//    offsets.
//  * Pair emission is atomic-free: each wave appends its pairs to a private
//    staging segment with a ballot + mbcnt prefix; each pair carries its rank
//    within its (row, slice).  k_scan_blocks and k_pairs_scatter turn counts
//    into canonical positions (i ascending, j ascending).  A wave whose segment
//    overflows is recomputed exactly by k_pairs_scatter.
#include "genga_internal.h"
#include <algorithm>

#include "device_common.h"

namespace genga {

struct KickDev {
    const double *x, *y, *z, *m, *rc;
    int64_t n;            // bodies (all systems)
    int64_t npad;
    // tiles: explicit list (batched) or implicit (single system)
    const TileDesc *tiles;
    int64_t ntiles;
    int gx;               // implicit: row blocks
    int64_t slice_len;    // implicit: columns per slice
    int tp;               // implicit, test-particle mode 1 or 2 (0: all bodies interact)
    int64_t nm;           // test-particle modes: bodies [0, nm) are massive
    int gx_m, s_m, gx_t;  // test-particle modes: massive / test-particle tiling
    int64_t len_m, len_t;
    int64_t mpad;         // test-particle modes: row stride of the massive rows' partials
    double *part;         // [slices][3][npad] (mixed: [slices][4][npad], 4th = sum m/r^2)
    int32_t *cnt;         // [slices][npad]
    int32_t *stage;       // [nwaves][WSEG][3]
    int32_t *wcount;      // [nwaves]
    int32_t *status;
    int32_t *queue;       // batch: next tile to take (reset to 0 by k_kick_reduce)
    int32_t *refine_cnt;  // mixed: rows listed for binary64 evaluation (reset here)
    int emit;
    double c15, c1875;    // 3/2 and 15/8
    double c53;           // 5/3
    double widen;         // mixed: squared widening of the binary32 pre-check radius
};

// Where the partial values of row i live: value c of slice s is at
// base + (s * ps + c) * stride + i.  In the test-particle modes the massive
// rows [0, nm) use a compact block of row stride mpad (they are few and may
// have many slices), followed by the test particles' slices of stride npad.
struct PartRows {
    size_t base, stride;
};

__device__ __forceinline__ PartRows part_rows(int tp, int64_t nm, int64_t mpad, int s_m,
                                              int64_t npad, int ps, int64_t i)
{
    if (!tp) return {0, (size_t)npad};
    if (i < nm) return {0, (size_t)mpad};
    return {(size_t)s_m * ps * mpad, (size_t)npad};
}

// Tile t: from the list, or from the implicit (row block, slice) grid.
template <int NT, int IPT>
__device__ __forceinline__ TileDesc get_tile(const KickDev &a, int64_t t)
{
    if (a.tiles) return a.tiles[t];
    TileDesc d;
    d.sys = 0;
    if (a.tp) {
        // massive rows against every column, then test-particle rows against
        // the massive columns only
        const int64_t tm = (int64_t)a.gx_m * a.s_m;
        if (t < tm) {
            const int64_t bx = t % a.gx_m, by = t / a.gx_m;
            d.row0 = bx * (int64_t)(NT * IPT);
            d.nrows = (int32_t)min((int64_t)(NT * IPT), a.nm - d.row0);
            d.slice = (int32_t)by;
            d.col0 = by * a.len_m;
            d.ncols = (int32_t)min(a.len_m, a.n - d.col0);
        } else {
            const int64_t u = t - tm;
            const int64_t bx = u % a.gx_t, by = u / a.gx_t;
            d.row0 = a.nm + bx * (int64_t)(NT * IPT);
            d.nrows = (int32_t)min((int64_t)(NT * IPT), a.n - d.row0);
            d.slice = (int32_t)by;
            d.col0 = by * a.len_t;
            d.ncols = (int32_t)min(a.len_t, a.nm - d.col0);
        }
        return d;
    }
    const int64_t bx = t % a.gx, by = t / a.gx;
    d.row0 = bx * (int64_t)(NT * IPT);
    d.nrows = (int32_t)min((int64_t)(NT * IPT), a.n - d.row0);
    d.slice = (int32_t)by;
    d.col0 = by * a.slice_len;
    d.ncols = (int32_t)min(a.slice_len, a.n - d.col0);
    return d;
}

// Kick variants sharing one kernel body.
enum KickMode : int {
    KM_F64 = 0,    // binary64 pair arithmetic
    KM_MIXED = 1,  // binary32 pair arithmetic on binary64 differences
    KM_PAIRS = 2,  // encounter list only (no forces)
};

// Per-lane state of the kick: IPT rows per lane.
template <int IPT>
struct Rows {
    double xi[IPT], yi[IPT], zi[IPT], rc2i[IPT];
    double iri[IPT];                     // 1 / rc_i
    double ax[IPT], ay[IPT], az[IPT];
    float rc2fi[IPT];                    // mixed: widened binary32 pre-check radius
    float axf[IPT], ayf[IPT], azf[IPT];  // mixed: binary32 partial sums
    float magf[IPT];                     // mixed: binary32 partial sum of m_j / r^2 (far pairs)
    double mag[IPT];                     // mixed: its binary64 accumulator
    int64_t ii[IPT];
    int kc[IPT];
};

// Rare path of one interaction: self pair, coincident bodies, changeover band
// (K < 1) and encounter-pair recording.  r2 is the exact binary64 squared
// separation, rc2j = rc_j^2 and irj = 1 / rc_j.  Returns the weight
// m_j K / r^3; a lane outside rho_ij keeps the fast path's weight sc_fast, so
// a result never depends on which lanes a (conservative) gate sent here.  1/r comes from v_rsq_f64 with one Newton correction
// (relative error below 5e-15); with 1/rho = min(1/rc_i, 1/rc_j) (division
// is monotone, so this is exactly fl(1 / max(rc_i, rc_j))) the band variable
// is y = (r/rho) / 0.9 - 1/9.  No global memory is read on this path.
template <int IPT, bool FORCES>
__device__ __forceinline__ double slow_pair(const KickDev &a, Rows<IPT> &R, int q, int64_t jg,
                                            double r2, double rc2j, double irj, double mj,
                                            double sc_fast, int64_t wave_g, int *wcnt)
{
    bool emit = false;
    double wk = 0.0;
    if (jg != R.ii[q]) {
        if (r2 == 0.0) {
            atomicOr(a.status, ST_NONFINITE);
        } else {
            const double rho2 = R.rc2i[q] > rc2j ? R.rc2i[q] : rc2j;
            const bool inside = r2 < rho2;
            emit = inside && (jg > R.ii[q]);
            if (FORCES) {
                wk = sc_fast;
                if (inside) {
                    const double y = __builtin_amdgcn_rsq(r2);
                    const double e = __builtin_fma(-r2, y * y, 1.0);
                    const double yc = __builtin_fma(y * e, 0.5, y);
                    const double irho = R.iri[q] < irj ? R.iri[q] : irj;
                    const double K =
                        changeover_of_y(__builtin_fma((r2 * yc) * irho, 1.0 / 0.9, -1.0 / 9.0));
                    wk = (mj * K) * (yc * yc * yc);
                }
            }
        }
    }
    if (a.emit) {
        const uint64_t mask = __ballot(emit);
        if (mask != 0ull) {
            // wave-private LDS counter: plain ds_read / ds_write (relaxed,
            // wavefront scope), so the compiler may still pipeline the tile reads
            const int base = __hip_atomic_load(wcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            if (emit) {
                const int pos = base + __popcll(mask & lanemask_lt());
                if (pos < WSEG) {
                    int32_t *e3 = a.stage + ((size_t)wave_g * WSEG + pos) * 3;
                    e3[0] = (int32_t)R.ii[q];
                    e3[1] = (int32_t)jg;
                    e3[2] = R.kc[q];
                }
                R.kc[q] += 1;
            }
            const uint64_t act = __ballot(1);
            if ((int)__lane_id() == __ffsll((unsigned long long)act) - 1)
                __hip_atomic_store(wcnt, base + __popcll(mask), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
    return wk;
}

// Mixed mode: pairs closer than MIXED_NEAR rho_ij are summed in binary64.  The
// largest binary32 terms are those of near neighbours; moving pairs inside
// 3 rho to binary64 keeps the per-acceleration error of the 0.5-4 AU disks
// below 1e-6 even for bodies whose net acceleration is 50-90 times smaller
// than the sum of the magnitudes of its terms.
constexpr double MIXED_NEAR = 3.0;
// Rows whose binary32 terms sum (in magnitude) to more than MIXED_KAPPA times
// the magnitude of their total are evaluated again in binary64: the binary32
// terms carry relative errors of a few 2^-24, so without this the error of a
// strongly cancelling row grows with that ratio.  The error per unit of the
// ratio depends on the arrangement: below 3e-8 on the disks (measured
// without the refinement: initial disks of 16,384-65,536 bodies and after
// 10-1000 steps), about 1.6e-7 for the bodies of a ring of equal masses,
// where rounding errors add coherently; hence 10.
constexpr double MIXED_KAPPA = 10.0;
constexpr int FOLD = 64;   // columns per binary32 partial sum (mixed mode)

// One column j against the lane's rows (the hot loop body).
//   b = (x_j, y_j, z_j, 3/2 m_j) for KM_F64, (x_j, y_j, z_j, m_j) for KM_PAIRS,
//   (x_j, y_j, z_j, {m_j, rc2f_j}) for KM_MIXED; *mj64 = m_j, *rc2j64 = rc_j^2.
//   gate2 (KM_F64, KM_PAIRS): a bound on r^2, at least max(rc_i^2, rc_j^2) for
//   every row of the lane, below which a pair takes the rare path, where the
//   exact test is made.
template <int IPT, int MODE>
__device__ __forceinline__ void interact(const KickDev &a, Rows<IPT> &R, const double4 b,
                                         const double gate2, const int64_t jg, const double c15,
                                         const double c1875, const double c53, const int64_t wave_g,
                                         int *wcnt, const double *rc2j64,
                                         const double *mj64, const double *irj64)
{
    if (MODE == KM_MIXED) {
        const float mjf = __int_as_float(__double2loint(b.w));
        const float rc2fj = __int_as_float(__double2hiint(b.w));
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const double dx = b.x - R.xi[q];
            const double dy = b.y - R.yi[q];
            const double dz = b.z - R.zi[q];
            const float dxf = (float)dx, dyf = (float)dy, dzf = (float)dz;
            const float r2f = __builtin_fmaf(dzf, dzf, __builtin_fmaf(dyf, dyf, dxf * dxf));
            // conservative binary32 test for "closer than MIXED_NEAR rho_ij"
            const bool near = r2f <= vmax_f32(R.rc2fi[q], rc2fj);
            const float yv = __builtin_amdgcn_rsqf(r2f);
            float mt = mjf * (yv * yv);   // magnitude m_j / r^2 of the binary32 term
            float sc = mt * yv;
            if (near) {
                // near pairs are evaluated in binary64; those inside rho_ij
                // (and the self pair, whose binary32 values are infinite)
                // take the changeover / encounter path
                sc = 0.0f;
                mt = 0.0f;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double mj = *mj64;
                const double rc2j_ = *rc2j64;
                double wk;
                const double y = __builtin_amdgcn_rsq(r2);
                const double yy = y * y;
                const double e = __builtin_fma(-r2, yy, 1.0);
                const double p = __builtin_fma(e, c1875, c15);
                const double my3 = mj * (yy * y);
                wk = __builtin_fma(my3 * e, p, my3);
                if (r2 <= vmax_f64(R.rc2i[q], rc2j_))
                    wk = slow_pair<IPT, true>(a, R, q, jg, r2, rc2j_, *irj64, mj, wk, wave_g, wcnt);
                R.ax[q] = __builtin_fma(dx, wk, R.ax[q]);
                R.ay[q] = __builtin_fma(dy, wk, R.ay[q]);
                R.az[q] = __builtin_fma(dz, wk, R.az[q]);
            }
            R.axf[q] = __builtin_fmaf(dxf, sc, R.axf[q]);
            R.ayf[q] = __builtin_fmaf(dyf, sc, R.ayf[q]);
            R.azf[q] = __builtin_fmaf(dzf, sc, R.azf[q]);
            R.magf[q] += mt;
        }
        return;
    }
    constexpr bool FORCES = MODE == KM_F64;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const double dx = b.x - R.xi[q];
        const double dy = b.y - R.yi[q];
        const double dz = b.z - R.zi[q];
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        // candidate: possibly inside the pair critical radius, or the self pair
        const bool cand = r2 <= gate2;
        double sc = 0.0;
        if (FORCES) {
            // m r^-3 from v_rsq_f64 (measured relative error below 2^-24):
            // with e = 1 - r2 y^2 (|e| < 1.1e-7), r2^{-3/2} = y^3 (1 - e)^{-3/2}
            //   = y^3 (1 + 3/2 e) + (15/8 e^2 < 2.3e-14) y^3 + ...
            // The first-order form leaves each term at most 2.3e-14 small;
            // over a whole disk that moves accelerations by < 2e-14 relative.
            // It is evaluated as (3/2 m) y^3 (5/3 - r2 y^2), with 3/2 m staged
            // in the tile, which takes one instruction less than
            // m y^3 + 3/2 e m y^3.
            const double yv = __builtin_amdgcn_rsq(r2);
            const double y2 = yv * yv;
            const double p = __builtin_fma(-r2, y2, c53);
            const double y3 = y2 * yv;
            sc = (b.w * y3) * p;
        }
        if (cand)
            sc = slow_pair<IPT, FORCES>(a, R, q, jg, r2, *rc2j64, *irj64, *mj64, sc, wave_g, wcnt);
        if (FORCES) {
            R.ax[q] = __builtin_fma(dx, sc, R.ax[q]);
            R.ay[q] = __builtin_fma(dy, sc, R.ay[q]);
            R.az[q] = __builtin_fma(dz, sc, R.az[q]);
        }
    }
}

// Mixed mode: add the binary32 partial sums into the binary64 accumulators.
template <int IPT, int MODE>
__device__ __forceinline__ void fold(Rows<IPT> &R)
{
    if (MODE != KM_MIXED) return;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        R.ax[q] += (double)R.axf[q];
        R.ay[q] += (double)R.ayf[q];
        R.az[q] += (double)R.azf[q];
        R.mag[q] += (double)R.magf[q];
        R.axf[q] = R.ayf[q] = R.azf[q] = R.magf[q] = 0.0f;
    }
}

// Shared-memory tile of one block: NT columns (one per thread per pass).
template <int NT>
struct KickSmem {
    double4 xyzm[NT];
    double rc2[NT];
    double m[NT];
    double irc[NT];     // 1 / rc_j
    double cmax[NT / 64];   // largest rc_j^2 among each staging wave's columns
    int wcnt[4];
};

// All rows of tile `td` against its columns; writes the slice partials, the
// per-row pair counts and the wave's staging count.
template <int NT, int IPT, int MODE>
__device__ __forceinline__ void process_tile(const KickDev &a, KickSmem<NT> &sm, const TileDesc &td,
                                             int64_t tile_index)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int64_t rowend = td.row0 + td.nrows;
    const int64_t rowbase = td.row0 + (int64_t)w * (64 * IPT);
    const int s = td.slice;
    const int64_t j0 = td.col0;
    const int64_t j1 = td.col0 + td.ncols;
    const int64_t wave_g = tile_index * (NT / 64) + w;
    // An opaque zero (mbcnt of an empty mask) marks values as per-lane, so the
    // compiler keeps the polynomial constants (not inline constants on gfx9)
    // and the LDS tile address in VGPRs instead of re-materialising them in
    // the hot loop.
    const int vzero = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
    const double c15 = a.c15 + (double)vzero, c1875 = a.c1875 + (double)vzero;
    const double c53 = a.c53 + (double)vzero;
    const double4 *t_xyzm = sm.xyzm + vzero;
    const double *t_rc2 = sm.rc2 + vzero;
    const double *t_m = sm.m + vzero;
    const double *t_irc = sm.irc + vzero;


    Rows<IPT> R;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int64_t slot = rowbase + q * 64 + lane;
        R.ii[q] = slot < rowend ? slot : -1;
        if (R.ii[q] >= 0) {
            R.xi[q] = a.x[R.ii[q]];
            R.yi[q] = a.y[R.ii[q]];
            R.zi[q] = a.z[R.ii[q]];
            const double r = a.rc[R.ii[q]];
            R.rc2i[q] = r * r;
            R.iri[q] = 1.0 / r;
        } else {
            // rows past the end: NaN positions never enter the slow path
            R.xi[q] = R.yi[q] = R.zi[q] = __builtin_nan("");
            R.rc2i[q] = 0.0;
            R.iri[q] = 0.0;
        }
        R.rc2fi[q] = (float)(R.rc2i[q] * a.widen);
        R.ax[q] = R.ay[q] = R.az[q] = R.mag[q] = 0.0;
        R.axf[q] = R.ayf[q] = R.azf[q] = R.magf[q] = 0.0f;
        R.kc[q] = 0;
    }
    // Binary64 and pair-list gate: a pair can be inside max(rc_i, rc_j) only
    // if r^2 is at most the largest rc^2 among the wave's rows and the tile's
    // columns, so one compare against that wave-uniform bound replaces the
    // per-pair max and compare (the rare path takes the exact test).
    double rg = 0.0;
    if (MODE != KM_MIXED) {
#pragma unroll
        for (int q = 0; q < IPT; ++q) rg = __builtin_fmax(rg, R.rc2i[q]);
        rg = wave_uniform(wave_max(rg));
    }
    int *wcnt = &sm.wcnt[w];
    if (lane == 0) __hip_atomic_store(wcnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);

    for (int64_t t0 = j0; t0 < j1; t0 += NT) {
        __syncthreads();
        {
            const int q = tid;
            const int64_t jg = t0 + q;
            double g = 0.0;
            if (jg < j1) {
                const double rcj = a.rc[jg];
                if (!(rcj >= 0.0 && rcj < INFINITY)) atomicOr(a.status, ST_RCRIT);
                // test-particle mode 1: a test particle acts on no body (it is
                // still tested for encounters with the massive rows)
                const double mj = (a.tp == 1 && jg >= a.nm) ? 0.0 : a.m[jg];
                if (MODE == KM_MIXED) {
                    const float rc2f = (float)(rcj * rcj * a.widen);
                    sm.xyzm[q] = make_double4(a.x[jg], a.y[jg], a.z[jg], pack_f32x2((float)mj, rc2f));
                    sm.m[q] = mj;
                } else {
                    sm.xyzm[q] = make_double4(a.x[jg], a.y[jg], a.z[jg],
                                              MODE == KM_F64 ? 1.5 * mj : mj);
                    sm.m[q] = mj;
                }
                sm.rc2[q] = rcj * rcj;
                if (MODE != KM_PAIRS) sm.irc[q] = 1.0 / rcj;
                g = rcj * rcj;
            }
            if (MODE != KM_MIXED) {
                const double gm = wave_max(g);
                if (lane == 0) sm.cmax[w] = gm;
            }
        }
        __syncthreads();
        double g2 = 0.0;
        if (MODE != KM_MIXED) {
            g2 = rg;
#pragma unroll
            for (int v = 0; v < NT / 64; ++v) g2 = __builtin_fmax(g2, sm.cmax[v]);
            g2 = wave_uniform(g2);
        }
        const int tn = (int)min((int64_t)NT, j1 - t0);
        int jj = 0;
        for (; jj + 4 <= tn; jj += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                interact<IPT, MODE>(a, R, t_xyzm[jj + u], g2, t0 + jj + u, c15, c1875, c53,
                                    wave_g, wcnt, t_rc2 + jj + u, t_m + jj + u, t_irc + jj + u);
            if ((jj & (FOLD - 1)) == FOLD - 4) fold<IPT, MODE>(R);
        }
        for (; jj < tn; ++jj)
            interact<IPT, MODE>(a, R, t_xyzm[jj], g2, t0 + jj, c15, c1875, c53, wave_g, wcnt,
                                t_rc2 + jj, t_m + jj, t_irc + jj);
        fold<IPT, MODE>(R);
    }

    constexpr int PS = MODE == KM_MIXED ? 4 : 3;
    // (a tile's rows are all massive or all test particles)
    const PartRows pr = part_rows(a.tp, a.nm, a.mpad, a.s_m, a.npad, PS, td.row0);
    const PartRows cr = part_rows(a.tp, a.nm, a.mpad, a.s_m, a.npad, 1, td.row0);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (R.ii[q] >= 0) {
            if (MODE != KM_PAIRS) {
                double *p = a.part + pr.base + (size_t)s * PS * pr.stride + R.ii[q];
                p[0] = R.ax[q];
                p[pr.stride] = R.ay[q];
                p[2 * pr.stride] = R.az[q];
                if (MODE == KM_MIXED) p[3 * pr.stride] = R.mag[q];
            }
            if (a.emit) a.cnt[cr.base + (size_t)s * cr.stride + R.ii[q]] = R.kc[q];
        }
    }
    if (a.emit && lane == 0)
        a.wcount[wave_g] = __hip_atomic_load(wcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// One tile per block (single system: grid = row blocks x column slices).
template <int NT, int IPT, int MODE>
__global__ __launch_bounds__(NT) void k_kick(KickDev a)
{
    __shared__ KickSmem<NT> sm;
    const int64_t t = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (MODE == KM_MIXED && t == 0 && threadIdx.x == 0) *a.refine_cnt = 0;
    process_tile<NT, IPT, MODE>(a, sm, get_tile<NT, IPT>(a, t), t);
}

// Persistent grid over a tile list (batched systems), sized to the blocks
// the chip holds at once: each block takes the next tile of the list (sorted
// by decreasing cost) from a device counter until the list is exhausted.
// Which block runs a tile does not change any result: every tile writes its
// own partial-sum and staging slots.
template <int NT, int IPT, int MODE>
__global__ __launch_bounds__(NT) void k_kick_persistent(KickDev a)
{
    __shared__ KickSmem<NT> sm;
    __shared__ int next;
    if (MODE == KM_MIXED && blockIdx.x == 0 && threadIdx.x == 0) *a.refine_cnt = 0;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.queue, 1);
        __syncthreads();
        const int64_t t = next;
        __syncthreads();
        if (t >= a.ntiles) break;
        process_tile<NT, IPT, MODE>(a, sm, a.tiles[t], t);
    }
}

// Sum the slice partials in slice order, apply v += h a, prepare pair offsets.
struct ReduceDev {
    double *part;
    int32_t *cnt;
    int32_t *rowloc;
    int64_t *bsum;
    double *vx, *vy, *vz;
    double *ax, *ay, *az;
    int32_t *status;
    int64_t n, npad;
    int slices;                   // single system
    const int32_t *sysid;         // batched: system of each body (else null)
    const int32_t *sys_slices;    // batched: column slices per system
    const double *sys_dt;         // batched: time step per system
    double G, h, hfac;            // v += h a (single) or hfac * dt_s * a (batched)
    int forces, emit;
    int tp;                       // test-particle mode: rows [0, nm) use s_m slices, the rest s_t
    int64_t nm, mpad;
    int s_m, s_t;
    int m_folded;                 // massive rows' sums already folded into their slice 0
    int32_t *queue;               // batch: tile counter of the kick, reset here
    double *px, *py, *pz;         // Sun kick fused after the velocities (hc_part non-null)
    const double *hc_part;
    int64_t hc_nb;
    double hc_h, hc_m_star;
    int pstride;                  // partial values per row and slice (3; mixed 4)
    int sym;                      // symmetric kick: row sums per tile, then column sums
    SymShape sh;
    const double *colpart;
    const double *fold;           // symmetric kick, small n: [SYM_FOLD][pstride][npad] part sums
                                  // (k_sym_fold), else null
    const SymSys *symb_sys;       // symmetric kick of a batch: per-system shapes, else null
    double kappa2;                // mixed: square of the refinement threshold (else 0)
    int32_t *refine_list, *refine_cnt;
};

// Symmetric kick, small n (few rows per block of the reduction): the sum of
// row i's values -- its group's tile sums in slice order, then the column sums
// of groups 0..g(i) in group order -- cut into SYM_FOLD contiguous parts, one
// thread per (part, component, row), so that the whole chip shares the loads;
// k_kick_reduce adds the parts in order (the same bits on every run).
struct SymFoldDev {
    const double *rowpart, *colpart;
    double *fold;
    SymShape sh;
    int ps;
    int64_t npad;
};

__global__ __launch_bounds__(RB) void k_sym_fold(SymFoldDev f)
{
    const int64_t idx = (int64_t)blockIdx.x * RB + threadIdx.x;
    const int64_t per = (int64_t)f.ps * f.npad;
    const int k = (int)(idx / per);
    const int c = (int)((idx % per) / f.npad);
    const int64_t i = idx % f.npad;
    if (k >= SYM_FOLD || i >= f.sh.n) return;
    const int64_t g = i / SYM_RG;
    const int64_t ns = f.sh.ns(g), len = ns + g + 1;
    const int64_t e0 = len * k / SYM_FOLD, e1 = len * (k + 1) / SYM_FOLD;
    const double *rp = f.rowpart + ((size_t)f.sh.tb(g) * f.ps + c) * SYM_RG + (i - g * SYM_RG);
    double acc = 0.0;
    int64_t e = e0;
    for (; e + 8 <= e1; e += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t q = e + u;
            if (q < ns) {
                v[u] = rp[(size_t)q * f.ps * SYM_RG];
            } else {
                const int64_t gg = q - ns;
                v[u] = f.colpart[(size_t)f.ps * f.sh.coloff(gg) + c * f.sh.collen(gg) +
                                 (i - gg * SYM_RG)];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; e < e1; ++e) {
        if (e < ns) {
            acc += rp[(size_t)e * f.ps * SYM_RG];
        } else {
            const int64_t gg = e - ns;
            acc += f.colpart[(size_t)f.ps * f.sh.coloff(gg) + c * f.sh.collen(gg) + (i - gg * SYM_RG)];
        }
    }
    f.fold[((size_t)k * f.ps + c) * f.npad + i] = acc;
}

// Symmetric kick: total of row i (group grp) over its nsl tiles and the
// column sums of groups 0..grp; components 0-2 into a3, component 3 (mixed:
// sum of m / r^2) into mag.
__device__ __forceinline__ void sym_row_total(const ReduceDev &r, const PartRows &pr, int nsl,
                                              int64_t grp, int64_t i, const SymShape &sh,
                                              const double *colpart, int64_t li, double a3[3],
                                              double &mag)
{
    const int nc = r.pstride;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double *p = r.part + pr.base + i;
    const size_t step = (size_t)nc * pr.stride;
    int s = 0;
    for (; s + 8 <= nsl; s += 8) {
        double v[8][4];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[k][c] = c < nc ? p[(size_t)(s + k) * step + c * pr.stride] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += v[k][c];
    }
    for (; s < nsl; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += c < nc ? p[(size_t)s * step + c * pr.stride] : 0.0;
    const int64_t ng = grp + 1;
    int64_t gg = 0;
    for (; gg + 8 <= ng; gg += 8) {
        double v[8][4];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t g2 = gg + k;
            const double *cp = colpart + (size_t)nc * sh.coloff(g2) + (li - g2 * SYM_RG);
            const int64_t L = sh.collen(g2);
#pragma unroll
            for (int c = 0; c < 4; ++c) v[k][c] = c < nc ? cp[c * L] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += v[k][c];
    }
    for (; gg < ng; ++gg) {
        const double *cp = colpart + (size_t)nc * sh.coloff(gg) + (li - gg * SYM_RG);
        const int64_t L = sh.collen(gg);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += c < nc ? cp[c * L] : 0.0;
    }
    a3[0] = acc[0];
    a3[1] = acc[1];
    a3[2] = acc[2];
    mag = acc[3];
}

__global__ __launch_bounds__(RB) void k_kick_reduce(ReduceDev r)
{
    __shared__ int64_t sm[RB / 64];
    __shared__ double hcs[3][RB];
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    const bool valid = i < r.n;
    double hcP[3] = {0.0, 0.0, 0.0};
    if (r.hc_part) {
        // P in the fixed order of k_hc_apply (every block the same)
        const int t = threadIdx.x;
        double p0 = 0.0, p1 = 0.0, p2 = 0.0;
        for (int64_t b = t; b < r.hc_nb; b += RB) {
            p0 += r.hc_part[b * 3 + 0];
            p1 += r.hc_part[b * 3 + 1];
            p2 += r.hc_part[b * 3 + 2];
        }
        hcs[0][t] = p0;
        hcs[1][t] = p1;
        hcs[2][t] = p2;
        __syncthreads();
        for (int hh = RB / 2; hh > 0; hh >>= 1) {
            if (t < hh) {
                hcs[0][t] += hcs[0][t + hh];
                hcs[1][t] += hcs[1][t + hh];
                hcs[2][t] += hcs[2][t + hh];
            }
            __syncthreads();
        }
        hcP[0] = hcs[0][0];
        hcP[1] = hcs[1][0];
        hcP[2] = hcs[2][0];
    }
    if (r.queue && i == 0) *r.queue = 0;
    int nsl = r.slices;
    if (r.tp) nsl = i < r.nm ? (r.m_folded ? 1 : r.s_m) : r.s_t;
    PartRows pr = part_rows(r.tp, r.nm, r.mpad, r.s_m, r.npad, r.pstride, i);
    PartRows cr = part_rows(r.tp, r.nm, r.mpad, r.s_m, r.npad, 1, i);
    double h = r.h;
    if (valid && r.sysid) {
        const int sy = r.sysid[i];
        nsl = r.sys_slices[sy];
        h = r.hfac * r.sys_dt[sy];
    }
    // symmetric kick: row i of its system (local index li, group grp), whose
    // tiles are stored from t0 on, slice by slice: [tile][pstride][SYM_RG]
    SymShape ssh = r.sh;
    const double *scol = r.colpart;
    int64_t li = i, so = 0, tbase = 0;
    if (r.sym && r.symb_sys && valid) {
        const SymSys ss = r.symb_sys[r.sysid[i]];
        ssh = ss.sh;
        so = ss.o;
        li = i - so;
        tbase = ss.tbase;
        scol = r.colpart + ss.cbase;
    }
    const int64_t grp = li / SYM_RG;
    if (r.sym) {
        nsl = (int)ssh.ns(grp);
        const int64_t t0 = tbase + ssh.tb(grp);
        // (non-negative: every system before this one has at least one tile per 512 bodies)
        pr = {(size_t)(t0 * r.pstride * SYM_RG - grp * SYM_RG - so), (size_t)SYM_RG};
        cr = {(size_t)(t0 * SYM_RG - grp * SYM_RG - so), (size_t)SYM_RG};
    }
    if (r.forces && valid) {
        double a3[3];
        double mag = 0.0;
        if (r.sym && r.fold) {
            // the SYM_FOLD part sums of k_sym_fold, in part order
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < SYM_FOLD; ++k)
                for (int c = 0; c < r.pstride; ++c)
                    acc[c] += r.fold[((size_t)k * r.pstride + c) * r.npad + i];
            a3[0] = acc[0];
            a3[1] = acc[1];
            a3[2] = acc[2];
            mag = acc[3];
        } else if (r.sym) {
            // row sums of the group's tiles in slice order, then the column
            // sums of the groups up to row i's in group order; the loads of
            // 8 tiles (groups) and all components are issued before their
            // additions, whose order is unchanged
            sym_row_total(r, pr, nsl, grp, i, ssh, scol, li, a3, mag);
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                a3[c] = ordered_sum(r.part + pr.base + c * pr.stride + i, r.pstride * pr.stride, nsl);
            if (r.kappa2 > 0.0)
                mag = ordered_sum(r.part + pr.base + 3 * pr.stride + i, r.pstride * pr.stride, nsl);
        }
        bool refine = false;
        if (r.kappa2 > 0.0) {
            // mixed: a row whose binary32 terms are large against their sum
            // (sum_j m_j / r^2 > kappa |sum_j m_j d / r^3|) is evaluated
            // again in binary64 by k_kick_refine
            const double a2 = a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2];
            refine = !(mag * mag <= r.kappa2 * a2);
        }
        if (refine) {
            r.refine_list[atomicAdd(r.refine_cnt, 1)] = (int32_t)i;
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) a3[c] *= r.G;
            if (!(isfinite(a3[0]) && isfinite(a3[1]) && isfinite(a3[2])))
                atomicOr(r.status, ST_NONFINITE);
            if (h != 0.0) {
                r.vx[i] = __builtin_fma(h, a3[0], r.vx[i]);
                r.vy[i] = __builtin_fma(h, a3[1], r.vy[i]);
                r.vz[i] = __builtin_fma(h, a3[2], r.vz[i]);
            }
            if (r.ax) {
                r.ax[i] = a3[0];
                r.ay[i] = a3[1];
                r.az[i] = a3[2];
            }
        }
    }
    if (r.hc_part && valid) {
        r.px[i] += (r.hc_h * hcP[0]) / r.hc_m_star;
        r.py[i] += (r.hc_h * hcP[1]) / r.hc_m_star;
        r.pz[i] += (r.hc_h * hcP[2]) / r.hc_m_star;
    }
    if (r.emit) {
        int64_t c = 0;
        if (valid) {
            int32_t *cp = r.cnt + cr.base + i;
            int s = 0;
            for (; s + 8 <= nsl; s += 8) {
                int32_t t[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) t[k] = cp[(size_t)(s + k) * cr.stride];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    cp[(size_t)(s + k) * cr.stride] = (int32_t)c;
                    c += t[k];
                }
            }
            for (; s < nsl; ++s) {
                const int32_t t = cp[(size_t)s * cr.stride];
                cp[(size_t)s * cr.stride] = (int32_t)c;
                c += t;
            }
        }
        int64_t tot;
        const int64_t ex = block_excl_scan<RB>(c, &tot, sm);
        if (valid) r.rowloc[i] = (int32_t)ex;
        if (threadIdx.x == 0) r.bsum[blockIdx.x] = tot;
    }
}

// Test-particle modes: one block per massive row folds its s_m slices into
// slice 0, so that k_kick_reduce reads one slice for these rows.  Thread t
// takes the slices [t ch, (t + 1) ch) in order, the FT thread sums are
// combined by a fixed tree in LDS; the pair counts become per-slice offsets
// within the row (a block exclusive scan in slice order), and slice 0 then
// holds the row total (its offset is 0, which k_kick_reduce writes back).
constexpr int FT = 256;

__global__ __launch_bounds__(FT) void k_fold_massive(ReduceDev r)
{
    __shared__ double sh[3][FT];
    __shared__ int64_t sc[FT / 64];
    const int64_t i = blockIdx.x;
    const int t = threadIdx.x;
    const int ns = r.s_m;
    const int ch = (ns + FT - 1) / FT;
    const int s0 = min(ns, t * ch), s1 = min(ns, s0 + ch);
    if (r.forces) {
        const PartRows pr = part_rows(r.tp, r.nm, r.mpad, r.s_m, r.npad, r.pstride, i);
        double *p = r.part + pr.base + i;
        const size_t step = (size_t)r.pstride * pr.stride;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            sh[c][t] = s1 > s0 ? ordered_sum(p + c * pr.stride + s0 * step, step, s1 - s0) : 0.0;
        __syncthreads();
        for (int h = FT / 2; h > 0; h >>= 1) {
            if (t < h) {
#pragma unroll
                for (int c = 0; c < 3; ++c) sh[c][t] += sh[c][t + h];
            }
            __syncthreads();
        }
        if (t == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) p[c * pr.stride] = sh[c][0];
        }
    }
    if (r.emit) {
        const PartRows cr = part_rows(r.tp, r.nm, r.mpad, r.s_m, r.npad, 1, i);
        int32_t *cp = r.cnt + cr.base + i;
        int64_t mine = 0;
        for (int s = s0; s < s1; ++s) mine += cp[(size_t)s * cr.stride];
        int64_t total;
        int64_t off = block_excl_scan<FT>(mine, &total, sc);
        for (int s = s0; s < s1; ++s) {
            const int32_t c = cp[(size_t)s * cr.stride];
            if (s > 0) cp[(size_t)s * cr.stride] = (int32_t)off;
            off += c;
        }
        if (t == 0) cp[0] = (int32_t)total;
    }
}

// Mixed mode: binary64 kick of the rows listed by k_kick_reduce, with the
// arithmetic of the binary64 kick.  Batched systems: one block per row
// (threads stride over the row's system, then a fixed-order block sum).
// Single system: k_refine_rows / k_refine_sum below.  The grids are fixed
// (the row count is read on the device), so the launches can be captured.
struct RefineDev {
    const double *x, *y, *z, *m, *rc;
    double *vx, *vy, *vz;
    double *ax, *ay, *az;
    int64_t n;
    const int32_t *list, *count;
    const int32_t *sysid;          // batched (else null)
    const int64_t *sys_off;        // batched: system offsets
    const double *sys_dt;          // batched: time step per system
    double G, h, hfac;
    double c53;
    int32_t *status;
};

constexpr int FB = 256;   // threads per refine block

__global__ __launch_bounds__(FB) void k_kick_refine(RefineDev a)
{
    __shared__ double sm[3][FB / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int vzero = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
    const double c53 = a.c53 + (double)vzero;
    const int cnt = *a.count;
    for (int p = blockIdx.x; p < cnt; p += gridDim.x) {
        const int64_t i = a.list[p];
        int64_t c0 = 0, c1 = a.n;
        double h = a.h;
        if (a.sysid) {
            const int sy = a.sysid[i];
            c0 = a.sys_off[sy];
            c1 = a.sys_off[sy + 1];
            h = a.hfac * a.sys_dt[sy];
        }
        const double xi = a.x[i], yi = a.y[i], zi = a.z[i], rci = a.rc[i];
        const double rc2i = rci * rci;
        double sx = 0.0, sy_ = 0.0, sz = 0.0;
        for (int64_t j = c0 + threadIdx.x; j < c1; j += FB) {
            const double dx = a.x[j] - xi, dy = a.y[j] - yi, dz = a.z[j] - zi;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double rcj = a.rc[j];
            const double mj = a.m[j];
            double wk;
            if (r2 <= vmax_f64(rc2i, rcj * rcj)) {
                wk = 0.0;
                if (j != i && r2 > 0.0) {
                    const double r = __builtin_sqrt(r2);
                    double K = 1.0;
                    if (r2 < rho2_of(rci, rcj)) K = changeover_k(r, rci > rcj ? rci : rcj);
                    wk = mj * K / (r2 * r);
                }
                // coincident bodies are reported by the main kick
            } else {
                const double yv = __builtin_amdgcn_rsq(r2);
                const double y2 = yv * yv;
                const double q = __builtin_fma(-r2, y2, c53);
                wk = ((1.5 * mj) * (y2 * yv)) * q;
            }
            sx = __builtin_fma(dx, wk, sx);
            sy_ = __builtin_fma(dy, wk, sy_);
            sz = __builtin_fma(dz, wk, sz);
        }
        for (int off = 32; off >= 1; off >>= 1) {
            sx += __shfl_xor(sx, off);
            sy_ += __shfl_xor(sy_, off);
            sz += __shfl_xor(sz, off);
        }
        if (lane == 0) {
            sm[0][w] = sx;
            sm[1][w] = sy_;
            sm[2][w] = sz;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a3[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double t = 0.0;
                for (int k = 0; k < FB / 64; ++k) t += sm[c][k];
                a3[c] = a.G * t;
            }
            if (!(isfinite(a3[0]) && isfinite(a3[1]) && isfinite(a3[2])))
                atomicOr(a.status, ST_NONFINITE);
            if (h != 0.0) {
                a.vx[i] = __builtin_fma(h, a3[0], a.vx[i]);
                a.vy[i] = __builtin_fma(h, a3[1], a.vy[i]);
                a.vz[i] = __builtin_fma(h, a3[2], a.vz[i]);
            }
            if (a.ax) {
                a.ax[i] = a3[0];
                a.ay[i] = a3[1];
                a.az[i] = a3[2];
            }
        }
        __syncthreads();
    }
}

// Single system: the listed rows in binary64.  A block takes a tile of 64
// listed rows (one per lane, every wave the same rows) and a block slice of
// the columns; its 4 waves split the slice in 4 contiguous parts, each staging
// 64 columns at a time in its own LDS region (no block barrier in the column
// loop), and their sums are added in wave order into the partial-sum region,
// [row tile][block slice][3][64]; k_refine_sum adds a row's block slices in
// order and applies v += h a.  The grids are fixed and the row count is read
// on the device, so the launches can be captured.
constexpr int RF_GRID = 2048;   // blocks of the refinement

struct RfSmem {
    double4 xyzm[4][64];   // (x, y, z, 3/2 m) of a wave's staged columns
    double rc2[4][64], m[4][64], irc[4][64];
    double acc[4][3][64];
};

// Row tiles, block slices and the block slice length (a multiple of 128
// columns: at least 32 per wave) for cnt listed rows; the partial sums fit
// cap doubles.
__device__ __forceinline__ void refine_split(int cnt, int64_t n, int64_t cap, int &RTn, int &SB,
                                             int64_t &blen)
{
    RTn = (cnt + 63) / 64;
    int64_t sb = RF_GRID / RTn;
    const int64_t most = cap / (192 * (int64_t)RTn);
    sb = sb < most ? sb : most;
    sb = sb > 1 ? sb : 1;
    blen = (((n + sb - 1) / sb) + 127) / 128 * 128;
    SB = (int)((n + blen - 1) / blen);
}

__global__ __launch_bounds__(256) void k_refine_rows(KickDev a, RefineDev f, int64_t cap)
{
    __shared__ RfSmem sm;
    const int cnt = *f.count;
    if (cnt == 0) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int RTn, SB;
    int64_t blen;
    refine_split(cnt, a.n, cap, RTn, SB, blen);
    const int items = RTn * SB;
    const int vzero = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
    const double c15 = a.c15 + (double)vzero, c1875 = a.c1875 + (double)vzero;
    const double c53 = a.c53 + (double)vzero;
    const double4 *t_xyzm = sm.xyzm[w] + vzero;
    const double *t_rc2 = sm.rc2[w] + vzero;
    const double *t_m = sm.m[w] + vzero;
    const double *t_irc = sm.irc[w] + vzero;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int rt = item / SB, sb = item % SB;
        const int pos = rt * 64 + lane;
        int64_t i = -1;
        Rows<1> R;
        R.xi[0] = R.yi[0] = R.zi[0] = __builtin_nan("");
        R.rc2i[0] = 0.0;
        R.iri[0] = 0.0;
        if (pos < cnt) {
            i = f.list[pos];
            R.xi[0] = a.x[i];
            R.yi[0] = a.y[i];
            R.zi[0] = a.z[i];
            const double r = a.rc[i];
            R.rc2i[0] = r * r;
            R.iri[0] = 1.0 / r;
        }
        R.ii[0] = i;
        R.ax[0] = R.ay[0] = R.az[0] = 0.0;
        R.kc[0] = 0;
        const int64_t q4 = blen / 4;
        const int64_t j0 = (int64_t)sb * blen + w * q4;
        const int64_t j1 = j0 + q4 < a.n ? j0 + q4 : a.n;
        for (int64_t t0 = j0; t0 < j1; t0 += 64) {
            const int64_t jg = t0 + lane;
            if (jg < j1) {
                const double mj = a.m[jg], rcj = a.rc[jg];
                sm.xyzm[w][lane] = make_double4(a.x[jg], a.y[jg], a.z[jg], 1.5 * mj);
                sm.m[w][lane] = mj;
                sm.rc2[w][lane] = rcj * rcj;
                sm.irc[w][lane] = 1.0 / rcj;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int tn = (int)(j1 - t0 < 64 ? j1 - t0 : 64);
            for (int jj = 0; jj < tn; ++jj)
                interact<1, KM_F64>(a, R, t_xyzm[jj], vmax_f64(R.rc2i[0], t_rc2[jj]), t0 + jj, c15,
                                    c1875, c53, 0, nullptr, t_rc2 + jj, t_m + jj, t_irc + jj);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        sm.acc[w][0][lane] = R.ax[0];
        sm.acc[w][1][lane] = R.ay[0];
        sm.acc[w][2][lane] = R.az[0];
        __syncthreads();
        if (w == 0) {
            double *P = a.part + ((size_t)rt * SB + sb) * 192;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                P[c * 64 + lane] = ((sm.acc[0][c][lane] + sm.acc[1][c][lane]) + sm.acc[2][c][lane]) +
                                   sm.acc[3][c][lane];
        }
        __syncthreads();
    }
}

// Sum each listed row's block-slice sums in slice order and apply v += h a:
// one wave per listed row, lanes take slices l, l + 64, ..., then a fixed
// xor-butterfly combines the lanes.
__global__ __launch_bounds__(RB) void k_refine_sum(KickDev a, RefineDev f, int64_t cap)
{
    const int cnt = *f.count;
    int RTn, SB;
    int64_t blen;
    refine_split(cnt, a.n, cap, RTn, SB, blen);
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (RB / 64);
    for (int64_t pos = (int64_t)blockIdx.x * (RB / 64) + (threadIdx.x >> 6); pos < cnt; pos += nw) {
        const int64_t i = f.list[pos];
        const double *P = a.part + (size_t)(pos / 64) * SB * 192 + (pos % 64);
        double a3[3] = {0.0, 0.0, 0.0};
        for (int s2 = lane; s2 < SB; s2 += 64) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a3[c] += P[(size_t)s2 * 192 + c * 64];
        }
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a3[c] += __shfl_xor(a3[c], off);
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a3[c] *= f.G;
            if (!(isfinite(a3[0]) && isfinite(a3[1]) && isfinite(a3[2])))
                atomicOr(f.status, ST_NONFINITE);
            if (f.h != 0.0) {
                f.vx[i] = __builtin_fma(f.h, a3[0], f.vx[i]);
                f.vy[i] = __builtin_fma(f.h, a3[1], f.vy[i]);
                f.vz[i] = __builtin_fma(f.h, a3[2], f.vz[i]);
            }
            if (f.ax) {
                f.ax[i] = a3[0];
                f.ay[i] = a3[1];
                f.az[i] = a3[2];
            }
        }
    }
}

// Exclusive scan of the per-block pair counts (one block); writes the total.
__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t *bsum, int64_t nb, int64_t *count,
                                                      int64_t capacity, int32_t *status)
{
    __shared__ int64_t sm[16];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t k = base + threadIdx.x;
        const int64_t v = k < nb ? bsum[k] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<1024>(v, &tot, sm);
        if (k < nb) bsum[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (count) *count = carry;
        if (carry > capacity) atomicOr(status, ST_OVERFLOW);
    }
}

// Place staged pairs at their canonical positions; recompute overflowed waves.
struct ScatterDev {
    KickDev k;                      // tiles of the kick that staged the pairs
    const int32_t *rowloc;
    const int64_t *boff;
    int32_t *pi, *pj;
    int64_t capacity;
    int nt, ipt;                    // kick block size and rows per thread
};

template <int NT, int IPT>
__device__ void scatter_wave(const ScatterDev &d, int64_t wave_g)
{
    const int lane = threadIdx.x;
    const KickDev &a = d.k;
    const int64_t t = wave_g / (NT / 64);
    const int w = (int)(wave_g % (NT / 64));
    const TileDesc td = get_tile<NT, IPT>(a, t);
    const int s = td.slice;
    const int nst = a.wcount[wave_g];
    if (nst <= WSEG) {
        for (int e = lane; e < nst; e += 64) {
            const int32_t *e3 = a.stage + ((size_t)wave_g * WSEG + e) * 3;
            const int64_t i = e3[0];
            const PartRows cr = part_rows(a.tp, a.nm, a.mpad, a.s_m, a.npad, 1, i);
            const int64_t pos =
                d.boff[i / RB] + d.rowloc[i] + a.cnt[cr.base + (size_t)s * cr.stride + i] + e3[2];
            if (pos < d.capacity) {
                d.pi[pos] = e3[0];
                d.pj[pos] = e3[1];
            }
        }
        return;
    }
    // staging overflowed: rebuild this wave's rows over its column range
    const int64_t rowend = td.row0 + td.nrows;
    const int64_t rowbase = td.row0 + (int64_t)w * (64 * IPT);
    const int64_t j0 = td.col0;
    const int64_t j1 = td.col0 + td.ncols;
    for (int q = 0; q < IPT; ++q) {
        const int64_t slot = rowbase + q * 64 + lane;
        if (slot >= rowend) continue;
        const int64_t i = slot;
        const PartRows cr = part_rows(a.tp, a.nm, a.mpad, a.s_m, a.npad, 1, i);
        int64_t pos = d.boff[i / RB] + d.rowloc[i] + a.cnt[cr.base + (size_t)s * cr.stride + i];
        const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
        const double rci = a.rc[i];
        const double rc2i = rci * rci;
        for (int64_t j = (j0 > i + 1 ? j0 : i + 1); j < j1; ++j) {
            const double dx = a.x[j] - xi, dy = a.y[j] - yi, dz = a.z[j] - zi;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double rcj = a.rc[j];
            const double rc2j = rcj * rcj;
            const double rho2 = rc2i > rc2j ? rc2i : rc2j;
            if (r2 < rho2) {
                if (pos < d.capacity) {
                    d.pi[pos] = (int32_t)i;
                    d.pj[pos] = (int32_t)j;
                }
                ++pos;
            }
        }
    }
}

__global__ __launch_bounds__(64) void k_pairs_scatter(ScatterDev d)
{
    const int64_t wave_g = blockIdx.x;
    if (d.nt == 64) {
        if (d.ipt == 2) scatter_wave<64, 2>(d, wave_g);
        else scatter_wave<64, 1>(d, wave_g);
    } else {
        if (d.ipt == 2) scatter_wave<KB, 2>(d, wave_g);
        else scatter_wave<KB, 1>(d, wave_g);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Symmetric kick: columns per slice, the widest (up to SYM_RG) that still
// gives about 4096 tiles, so that row sums cost little HBM traffic while the
// chip holds several rounds of tiles (65,536 bodies: 512 columns, 8,256
// tiles; 128 and 256 columns measured within 0.3 % of its kick time, with
// longer reductions).
static int sym_width(int64_t n)
{
    int W = SYM_RG;
    while (W > 64 && sym_shape(n, W).T < 4096) W /= 2;
    return W;
}

KickCfg choose_kick_cfg(int64_t n, const genga_params *p)
{
    KickCfg c;
    c.ipt = (p && p->ipt > 0) ? p->ipt : 1;
    if (c.ipt != 1 && c.ipt != 2) c.ipt = 1;
    c.nt = KB;
    const int64_t rows_per_block = (int64_t)c.nt * c.ipt;
    c.gx = (int)((n + rows_per_block - 1) / rows_per_block);
    int64_t slices;
    if (p && p->slices > 0) {
        slices = p->slices;
    } else {
        // about 12288 blocks (48 per CU, ~10 waves of resident blocks): large
        // systems get column slices for latency hiding and a short tail, small
        // ones short slices so that no wave walks more than a few hundred
        // columns on an otherwise idle chip (measured at 65,536 bodies: 32,
        // 40, 48, 64 slices give 2.70, 2.65, 2.64, 2.66 ms)
        slices = (12288 + c.gx - 1) / c.gx;
    }
    if (slices < 1) slices = 1;
    // slices of a multiple of 64 columns (64 at the least)
    int64_t len = (n + slices - 1) / slices;
    len = ((len + 63) / 64) * 64;
    c.slice_len = len;
    c.slices = (int)((n + c.slice_len - 1) / c.slice_len);
    c.ntiles = (int64_t)c.gx * c.slices;
    c.gy = c.slices;
    if (p && p->tp_mode != 0 && p->n_massive < n) {
        // test particles: massive rows x all columns, test-particle rows x
        // massive columns, each class with about half of the blocks
        const int64_t nm = p->n_massive > 0 ? p->n_massive : 0;
        c.tp = p->tp_mode;
        c.nm = nm;
        c.gx_m = (int)((nm + rows_per_block - 1) / rows_per_block);
        c.gx_t = (int)((n - nm + rows_per_block - 1) / rows_per_block);
        auto split = [](int64_t cols, int gxc, int &sc, int64_t &len) {
            if (cols <= 0 || gxc <= 0) {
                sc = 0;
                len = 64;
                return;
            }
            int64_t want = (6144 + gxc - 1) / gxc;
            const int64_t most = (cols + 63) / 64;
            if (want > most) want = most;
            if (want < 1) want = 1;
            len = (((cols + want - 1) / want) + 63) / 64 * 64;
            sc = (int)((cols + len - 1) / len);
        };
        split(n, c.gx_m, c.s_m, c.len_m);
        split(nm, c.gx_t, c.s_t, c.len_t);
        c.ntiles = (int64_t)c.gx_m * c.s_m + (int64_t)c.gx_t * c.s_t;
        // the compact block of the massive rows (up to 5 values per slice, as
        // the kick's region is sized for) in npad-long slice rows
        const int64_t npad = ((n + RB - 1) / RB) * RB;
        c.mpad = ((nm + 63) / 64) * 64;
        c.slices = (int)(c.s_t + ((int64_t)c.s_m * c.mpad + npad - 1) / npad);
        if (c.slices < 1) c.slices = 1;
        c.gx = (int)c.ntiles;    // one-dimensional launch over the tile numbers
        c.gy = 1;
    }
    c.nwaves = c.ntiles * (c.nt / 64);
    // forces of one all-massive system (binary64 or mixed): the symmetric
    // kick from SYM_MIN_N bodies (or as the flags ask)
    const int flags = p ? p->flags : 0;
    const bool plain = !p || p->tp_mode == 0 || p->n_massive >= n;
    if (plain && !(flags & GENGA_FLAG_DIRECTED) &&
        (n >= SYM_MIN_N || (flags & GENGA_FLAG_SYMMETRIC))) {
        int W = sym_width(n);
        if (p && p->slices > 0) {
            // slices over a row group's own rows: 1, 2, 4, 8 or 16
            int dd = 1;
            while (dd * 2 <= p->slices && dd < SYM_RG / 64) dd *= 2;
            W = SYM_RG / dd;
        }
        const SymShape h = sym_shape(n, W);
        // its row and column sums (up to 5 per row and tile or group: the
        // adjoint's) grow as n^2 / SYM_RG: by default the symmetric form stays
        // within SYM_WS_MAX bytes of them
        const double bytes = 40.0 * ((double)h.T * SYM_RG + (double)h.coloff(h.G));
        if ((flags & GENGA_FLAG_SYMMETRIC) || bytes <= (double)SYM_WS_MAX) {
            c.use_sym = true;
            c.sym = h;
        }
    }
    return c;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Layout make_layout(int64_t n, const KickCfg &c, int64_t S)
{
    Layout L;
    L.npad = ((n + RB - 1) / RB) * RB;
    L.nb = (n + RB - 1) / RB;
    size_t off = 0;
    L.status = off;
    off += 256;
    // the symmetric kick's row sums [T][3 or 4][SYM_RG] and column sums (with
    // the row totals' parts below SYM_FOLD_BELOW bodies), or the symmetric
    // adjoint's 5 of each, share the partial-sum region; the kick's per-tile
    // pair counts the count region
    const size_t symx = (size_t)c.sym.T * SYM_RG + (size_t)c.sym.coloff(c.sym.G);
    const size_t sym_part =
        c.use_sym ? std::max(4 * symx + (n < SYM_FOLD_BELOW ? (size_t)SYM_FOLD * 4 * L.npad : 0),
                             5 * symx)
                  : 0;
    size_t sym_cnt = c.use_sym ? (size_t)c.sym.T * SYM_RG : 0;
    size_t nw = std::max<size_t>((size_t)c.nwaves, c.use_sym ? (size_t)c.sym.T * SYM_NW : 0);
    size_t symb_part = 0;
    if (c.use_symb) {
        symb_part = 3 * ((size_t)c.symb_T * SYM_RG + (size_t)c.symb_cols);
        sym_cnt = std::max(sym_cnt, (size_t)c.symb_T * SYM_RG);
        nw = std::max(nw, (size_t)c.symb_T * SYM_NW);
    }
    L.part = off;   // 3 values per row and slice for the kick, 5 for its adjoint
    off = align256(off + sizeof(double) * std::max({5 * (size_t)c.slices * L.npad, sym_part, symb_part}));
    L.cnt = off;
    off = align256(off + sizeof(int32_t) * std::max((size_t)c.slices * L.npad, sym_cnt));
    L.rowloc = off;
    off = align256(off + sizeof(int32_t) * (size_t)L.npad);
    L.bsum = off;
    off = align256(off + sizeof(int64_t) * (size_t)(L.nb + 1));
    L.stage = off;
    off = align256(off + sizeof(int32_t) * 3 * (size_t)WSEG * nw);
    L.wcount = off;
    off = align256(off + sizeof(int32_t) * nw);
    L.hc = off;
    off = align256(off + sizeof(double) * 3 * (size_t)L.nb);
    L.hc2 = off;
    off = align256(off + sizeof(double) * 3 * (size_t)L.nb);
    L.rlist = off;
    off = align256(off + sizeof(int32_t) * (size_t)L.npad);
    L.gru = off;
    off = align256(off + sizeof(double) * 3 * (size_t)L.npad);
    L.grp = off;
    off = align256(off + sizeof(double) * 4 * (size_t)L.nb);
    if (S > 0) {
        L.P = off;
        off = align256(off + sizeof(double) * 3 * (size_t)S);
        L.tiles = off;
        off = align256(off + sizeof(TileDesc) * (size_t)c.ntiles);
        L.sysid = off;
        off = align256(off + sizeof(int32_t) * (size_t)L.npad);
        L.sys_slices = off;
        off = align256(off + sizeof(int32_t) * (size_t)S);
        L.offsets = off;
        off = align256(off + sizeof(int64_t) * (size_t)(S + 1));
        if (c.use_symb) {
            L.symsys = off;
            off = align256(off + sizeof(SymSys) * (size_t)S);
            L.symtiles = off;
            off = align256(off + sizeof(SymTileB) * (size_t)c.symb_T);
            L.symorder = off;
            off = align256(off + sizeof(int32_t) * (size_t)c.symb_T);
        }
    }
    L.total = off;
    return L;
}

template <int NT, int IPT, int MODE>
static void launch_k(const KickDev &d, const KickCfg &c, hipStream_t s)
{
    if (d.tiles)
        hipLaunchKernelGGL((k_kick_persistent<NT, IPT, MODE>), dim3(c.grid), dim3(NT), 0, s, d);
    else
        hipLaunchKernelGGL((k_kick<NT, IPT, MODE>), dim3(c.gx, c.gy), dim3(NT), 0, s, d);
}

template <int NT, int IPT, int MODE>
static int occupancy_k()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_kick_persistent<NT, IPT, MODE>, NT, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

int kick_blocks_per_cu(const KickCfg &c, int precision)
{
    const bool mixed = precision == GENGA_MIXED;
    if (c.nt == 64) {
        if (c.ipt == 2) return mixed ? occupancy_k<64, 2, KM_MIXED>() : occupancy_k<64, 2, KM_F64>();
        return mixed ? occupancy_k<64, 1, KM_MIXED>() : occupancy_k<64, 1, KM_F64>();
    }
    if (c.ipt == 2) return mixed ? occupancy_k<KB, 2, KM_MIXED>() : occupancy_k<KB, 2, KM_F64>();
    return mixed ? occupancy_k<KB, 1, KM_MIXED>() : occupancy_k<KB, 1, KM_F64>();
}

template <int NT, int IPT>
static void launch_mode(const KickDev &d, const KickCfg &c, int mode, hipStream_t s)
{
    if (mode == KM_MIXED) launch_k<NT, IPT, KM_MIXED>(d, c, s);
    else if (mode == KM_PAIRS) launch_k<NT, IPT, KM_PAIRS>(d, c, s);
    else launch_k<NT, IPT, KM_F64>(d, c, s);
}

hipError_t launch_kick(const KickLaunch &k, const KickCfg &c, const Layout &L, char *ws,
                       hipStream_t s)
{
    KickDev d;
    d.x = k.x; d.y = k.y; d.z = k.z; d.m = k.m; d.rc = k.rc;
    d.n = k.n;
    d.npad = L.npad;
    d.tiles = k.tiles;
    d.ntiles = c.ntiles;
    d.gx = c.gx;
    d.slice_len = c.slice_len;
    d.tp = c.tp;
    d.nm = c.nm;
    d.gx_m = c.gx_m;
    d.s_m = c.s_m;
    d.gx_t = c.gx_t;
    d.len_m = c.len_m;
    d.len_t = c.len_t;
    d.mpad = c.mpad;
    d.part = (double *)(ws + L.part);
    d.cnt = (int32_t *)(ws + L.cnt);
    d.stage = (int32_t *)(ws + L.stage);
    d.wcount = (int32_t *)(ws + L.wcount);
    d.status = (int32_t *)(ws + L.status);
    d.queue = k.tiles ? (int32_t *)(ws + L.status) + 1 : nullptr;
    d.refine_cnt = (int32_t *)(ws + L.status) + 2;
    d.emit = k.pairs != nullptr;
    d.c15 = 1.5;
    d.c53 = 5.0 / 3.0;
    d.c1875 = 1.875;
    // Mixed mode evaluates every pair closer than MIXED_NEAR rho_ij in
    // binary64: the binary32 test uses (MIXED_NEAR rho)^2 with a relative
    // margin of 2^-14, far above the binary32 rounding of r^2 (< 2^-21), so
    // no pair inside rho_ij can be missed.
    d.widen = MIXED_NEAR * MIXED_NEAR * (1.0 + 0x1p-14);

    const int mode = !k.forces ? KM_PAIRS : (k.precision == GENGA_MIXED ? KM_MIXED : KM_F64);
    const bool refine = mode == KM_MIXED;
    const bool symb = c.use_symb && mode == KM_F64 && k.tiles;
    const bool sym = (c.use_sym && (mode == KM_F64 || mode == KM_MIXED) && !k.tiles && c.tp == 0) || symb;
    const int sym_ps = mode == KM_MIXED ? 4 : 3;
    const int64_t sym_T = symb ? c.symb_T : c.sym.T;
    SymBatch sb{nullptr, nullptr, nullptr, 0, 0};
    if (symb) {
        sb.sys = (const SymSys *)(ws + L.symsys);
        sb.tiles = (const SymTileB *)(ws + L.symtiles);
        sb.order = (const int32_t *)(ws + L.symorder);
        sb.S = c.symb_S;
        sb.T = c.symb_T;
    }
    if (k.ev0) {
        hipError_t e0 = hipEventRecord((hipEvent_t)k.ev0, s);
        if (e0 != hipSuccess) return e0;
    }
    if (symb) {
        hipError_t es = launch_kick_sym_b(sb, k.x, k.y, k.z, k.m, k.rc, d.part,
                                          d.part + (size_t)3 * sym_T * SYM_RG, d.cnt, d.stage,
                                          d.wcount, d.status, d.emit, s);
        if (es != hipSuccess) return es;
    } else if (sym) {
        hipError_t es = launch_kick_sym(c.sym, mode == KM_MIXED, d.widen, k.x, k.y, k.z, k.m,
                                        k.rc, d.part, d.part + (size_t)sym_ps * c.sym.T * SYM_RG,
                                        d.cnt, d.stage, d.wcount, d.status, d.refine_cnt,
                                        d.emit, s);
        if (es != hipSuccess) return es;
    } else if (c.ntiles == 0) {
        // (test-particle mode without massive bodies: nothing acts on anything)
    } else if (c.nt == 64) {
        if (c.ipt == 2) launch_mode<64, 2>(d, c, mode, s);
        else launch_mode<64, 1>(d, c, mode, s);
    } else {
        if (c.ipt == 2) launch_mode<KB, 2>(d, c, mode, s);
        else launch_mode<KB, 1>(d, c, mode, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (k.ev1 && !refine) {
        e = hipEventRecord((hipEvent_t)k.ev1, s);
        if (e != hipSuccess) return e;
    }

    ReduceDev r;
    r.part = d.part; r.cnt = d.cnt;
    r.rowloc = (int32_t *)(ws + L.rowloc);
    r.bsum = (int64_t *)(ws + L.bsum);
    r.vx = k.vx; r.vy = k.vy; r.vz = k.vz;
    r.ax = k.ax; r.ay = k.ay; r.az = k.az;
    r.status = d.status;
    r.n = k.n; r.npad = L.npad; r.slices = c.slices;
    r.sysid = k.sysid;
    r.sys_slices = k.sys_slices;
    r.sys_dt = k.sys_dt;
    r.G = k.G; r.h = k.h; r.hfac = k.hfac;
    r.forces = k.forces;
    r.emit = d.emit;
    r.queue = d.queue;
    r.tp = c.tp;
    r.nm = c.nm;
    r.s_m = c.s_m;
    r.s_t = c.s_t;
    r.mpad = c.mpad;
    r.m_folded = 0;
    r.px = k.px; r.py = k.py; r.pz = k.pz;
    r.hc_part = k.hc_part;
    r.hc_nb = k.hc_nb;
    r.hc_h = k.hc_h;
    r.hc_m_star = k.hc_m_star;
    r.pstride = refine ? 4 : 3;
    r.sym = sym ? 1 : 0;
    r.sh = c.sym;
    r.colpart = d.part + (size_t)sym_ps * sym_T * SYM_RG;
    r.symb_sys = symb ? sb.sys : nullptr;
    r.kappa2 = refine ? MIXED_KAPPA * MIXED_KAPPA : 0.0;
    r.refine_list = (int32_t *)(ws + L.rlist);
    r.refine_cnt = d.refine_cnt;
    r.fold = nullptr;
    if ((r.forces || r.emit) && c.tp && c.nm > 0 && c.s_m > 1) {
        hipLaunchKernelGGL(k_fold_massive, dim3((unsigned)c.nm), dim3(FT), 0, s, r);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        r.m_folded = 1;
    }
    if (sym && !symb && r.forces && k.n < SYM_FOLD_BELOW) {
        SymFoldDev f;
        f.rowpart = d.part;
        f.colpart = r.colpart;
        f.fold = d.part + (size_t)4 * ((size_t)c.sym.T * SYM_RG + (size_t)c.sym.coloff(c.sym.G));
        f.sh = c.sym;
        f.ps = sym_ps;
        f.npad = L.npad;
        const int64_t threads = (int64_t)SYM_FOLD * sym_ps * L.npad;
        hipLaunchKernelGGL(k_sym_fold, dim3((unsigned)((threads + RB - 1) / RB)), dim3(RB), 0, s, f);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        r.fold = f.fold;
    }
    if (r.forces || r.emit) {
        hipLaunchKernelGGL(k_kick_reduce, dim3((unsigned)L.nb), dim3(RB), 0, s, r);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (refine) {
        RefineDev f;
        f.x = k.x; f.y = k.y; f.z = k.z; f.m = k.m; f.rc = k.rc;
        f.vx = k.vx; f.vy = k.vy; f.vz = k.vz;
        f.ax = k.ax; f.ay = k.ay; f.az = k.az;
        f.n = k.n;
        f.list = r.refine_list;
        f.count = r.refine_cnt;
        f.sysid = k.sysid;
        f.sys_off = k.sys_off;
        f.sys_dt = k.sys_dt;
        f.G = k.G; f.h = k.h; f.hfac = k.hfac;
        f.c53 = 5.0 / 3.0;
        f.status = d.status;
        if (k.sysid) {
            // enough blocks for a few percent of the rows at one row per block
            const int64_t blocks = std::min<int64_t>(std::max<int64_t>(k.n, 1), 2048);
            hipLaunchKernelGGL(k_kick_refine, dim3((unsigned)blocks), dim3(FB), 0, s, f);
        } else {
            // the main kick's partial sums are consumed: reuse their region
            const int64_t cap = 5 * (int64_t)c.slices * L.npad;
            KickDev rd = d;
            rd.emit = 0;
            hipLaunchKernelGGL(k_refine_rows, dim3(RF_GRID), dim3(256), 0, s, rd, f, cap);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_refine_sum, dim3((unsigned)std::min<int64_t>(L.nb, 1024)),
                               dim3(RB), 0, s, rd, f, cap);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (k.ev1) {
            e = hipEventRecord((hipEvent_t)k.ev1, s);
            if (e != hipSuccess) return e;
        }
    }
    if (!d.emit) return hipSuccess;

    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, r.bsum, L.nb, k.pairs->count,
                       k.pairs->capacity, d.status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    if (sym)
        return launch_scatter_sym(c.sym, symb ? &sb : nullptr, k.x, k.y, k.z, k.rc, d.cnt, d.stage,
                                  d.wcount, r.rowloc, r.bsum, k.pairs, s);
    ScatterDev sd;
    sd.k = d;
    sd.rowloc = r.rowloc;
    sd.boff = r.bsum;
    sd.pi = k.pairs->i; sd.pj = k.pairs->j;
    sd.capacity = k.pairs->capacity;
    sd.nt = c.nt;
    sd.ipt = c.ipt;
    if (c.nwaves == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs_scatter, dim3((unsigned)c.nwaves), dim3(64), 0, s, sd);
    return hipGetLastError();
}

}  // namespace genga
