// Symmetric changeover-weighted kick (binary64, one system, every body massive):
// each unordered pair is evaluated once and its force applied to both bodies.
//
// Paper: GENGA II Sect. 2 (interaction part H_B of the democratic-heliocentric
// splitting, eq. Hb, whose pair terms G m_i m_j K / r_ij are symmetric in i and
// j when the pair's critical radius is max(rc_i, rc_j), eq. rcrit), Sect. 6.2
// (changeover band 0.1 < r/r_crit < 1 with the form of Chambers 1999 eq. 10),
// Appendix A (kick with the close-encounter pre-check), Appendix B (fixed
// order of the encounter list).
//
// Design for gfx950 (wave64, 256 CUs, FP64 vector ALU bound):
//  * Rows are cut into groups of SYM_RG = 512: one block of 4 waves with 2
//    rows per lane.  Group g works on the columns [g SYM_RG, n) -- its own rows
//    and every row after them -- in slices of W columns; a tile is one slice
//    (W = 512 at 65,536 bodies: 8,256 tiles; measured against 8-wave blocks of
//    1,024 rows and against W = 128, 256: 1.76 ms per kick, 2-7 % faster).
//  * A tile's columns are staged in LDS in chunks of 64, each stored twice in
//    a row so that lane l reads entry l + k at step k without a wrap.  At step
//    k (0..63) lane l takes column (l + k) mod 64: the 64 lanes of a wave meet
//    64 different columns, and each lane carries the running sum of the
//    column it is on.  After every step the three column sums move one lane
//    down (v_mov_b32_dpp wave_rol:1, lane l receives lane l + 1), which hands
//    each lane the sum of its next column; after 64 steps every sum is back
//    in the lane of its column.  Per step and lane: 2 pairs of 20 FP64
//    instructions (one of them v_rsq_f64) and 6 moves cover 4 directed
//    interactions (the one-sided kick spends 4 x 17).
//  * Chunks over the group's own rows: a chunk after the lane's row chunk is
//    done symmetrically, the row's own chunk one-sided (each lane sums all 64
//    columns into its row only, self pair excluded), a chunk before it not at
//    all: those pairs are transposes of pairs done symmetrically.
//  * The 4 waves' column sums of a chunk are added in LDS in wave order and
//    written once per (group, column); row sums once per (tile, row).
//    k_kick_reduce adds a row's tile sums in slice order, then its column
//    sums in group order: no atomics, the same bits on every run.
//  * Pairs inside the critical radius take a divergent rare path (K, the
//    self pair, coincident bodies, encounter recording) as in the one-sided
//    kick.  A lane meets its columns in rotated order, so a staged pair
//    carries no rank; k_pairs_scatter_sym ranks it among the pairs of its row
//    in the wave's staging segment, which hold all of that row's pairs of
//    the tile, and the list comes out in canonical order (i, then j).
#include "genga_internal.h"
#include <algorithm>

#include "device_common.h"
#include "sym_common.h"

namespace genga {

SymShape sym_shape(int64_t n, int W)
{
    SymShape h;
    h.n = n;
    h.W = W;
    h.d = SYM_RG / W;
    h.G = (n + SYM_RG - 1) / SYM_RG;
    h.S0 = (n + W - 1) / W;
    h.T = h.tb(h.G);
    h.tfull = h.bf(h.G - 1);
    return h;
}

struct SymDev {
    const double *x, *y, *z, *m, *rc;
    SymShape sh;
    double *rowpart;   // [T][ps][SYM_RG]
    double *colpart;   // group g: [ps][collen(g)] from ps coloff(g)
    int32_t *cnt;      // [T][SYM_RG]
    int32_t *stage;    // [T SYM_NW][WSEG][3]  (i, j, unused)
    int32_t *wcount;   // [T SYM_NW]
    int32_t *status;
    int32_t *refine_cnt;   // mixed: rows listed for binary64 evaluation (reset here)
    int64_t o;             // batch: the system's first body (x..rc and colpart are the
                           // system's; staged pairs carry global indices); else 0
    int emit;
    int ps;            // partial values per row: 3 (a), mixed 4 (a, sum of m / r^2)
    double c53;        // 5/3
    double c15, c1875; // 3/2, 15/8
    double widen;      // mixed: squared widening of the binary32 near test
    double far_row, far_col;   // coordinates of padding rows and columns
};

// Padding rows and columns sit far away, on opposite sides (no two padding
// bodies coincide), with mass 0 and critical radius 0: r^2 stays finite (below
// 1.3e37, also in binary32), every weight they give or take is 0 and they
// never reach the rare path.  (Passed as kernel arguments, so that they sit in
// scalar registers.)
constexpr double SYM_FAR_ROW = 1e18, SYM_FAR_COL = -1e18;

// One chunk of 64 columns, stored twice (entries e and e + 64 are column e).
template <bool MIXED>
struct SymCols;
template <>
struct SymCols<false> {
    double2 xy[128];
    double2 zm[128];   // (z, 3/2 m)
    double rc2[128];
    double m[128];
};
template <>
struct SymCols<true> {
    double2 xy[128];
    double z[128];
    float2 fw[128];    // (m, widened rc^2) in binary32
    double rc2[128];
    double m[128];
};

template <bool MIXED>
struct SymSmem {
    SymCols<MIXED> col[2];
    double acc[2][MIXED ? 4 : 3][SYM_NW][64];   // column sums of a chunk, per wave
    double nacc[MIXED ? SYM_NW : 1][3][64];      // mixed: binary64 column sums of near pairs
    int gmax[2];       // binary64: high word of a bound of the largest rc^2 among
                       // the columns of chunk b (wave_max_hi)
    int wcnt[SYM_NW];
};

template <bool MIXED>
struct SymRows {
    double xi[SYM_IPT], yi[SYM_IPT], zi[SYM_IPT], rc2i[SYM_IPT];
    double mw[SYM_IPT];    // 3/2 m_i (mixed: m_i)
    double ax[SYM_IPT], ay[SYM_IPT], az[SYM_IPT];
    int ii[SYM_IPT];       // row index, -1 for padding (n < 2^31)
    int kc[SYM_IPT];
    // mixed
    double mag[SYM_IPT];                  // binary64 sum of the binary32 m_j / r^2
    float rc2fi[SYM_IPT], mif[SYM_IPT];
    float axf[SYM_IPT], ayf[SYM_IPT], azf[SYM_IPT], magf[SYM_IPT];
};

// Rare path of one pair (binary64: r^2 at most the wave's gate bound, which is
// at least max(rc_i^2, rc_j^2); mixed: r^2 <= max(rc_i^2, rc_j^2)): the self pair, coincident bodies, the changeover band
// and encounter recording.  si, sj hold the fast weights (m_j and m_i times
// r^-3) and are replaced by K-weighted ones inside rho_ij; a pair at or beyond
// rho_ij keeps them (K = 1) and is not recorded.  1/r and 1/rho from
// v_rsq_f64 with one Newton correction (relative error below 5e-15), so the
// band variable is y = (r/rho) / 0.9 - 1/9; in the binary64 kick m_i is
// (2/3) (3/2 m_i), to 2 ulp.  Whether a pair is inside rho_ij, and so in the
// encounter list, is decided by r^2 < max(rc_i^2, rc_j^2) alone.
template <bool MIXED>
__device__ __forceinline__ void sym_slow(const SymDev &a, SymRows<MIXED> &R, int q, int jg,
                                         double r2, double rc2c, double mc, double &si,
                                         double &sj, int64_t wave_g, int *wcnt)
{
    bool emit = false;
    if (jg == R.ii[q]) {
        si = 0.0;
        sj = 0.0;
    } else if (r2 == 0.0) {
        atomicOr(a.status, ST_NONFINITE);
        si = 0.0;
        sj = 0.0;
    } else {
        const double rho2 = R.rc2i[q] > rc2c ? R.rc2i[q] : rc2c;
        const bool inside = r2 < rho2;
        emit = inside && jg > R.ii[q];
        if (inside) {
            const double yc = rsq_nr(r2);
            const double irho = rsq_nr(rho2);
            const double K = changeover_of_y(__builtin_fma((r2 * yc) * irho, 1.0 / 0.9, -1.0 / 9.0));
            const double kr = K * (yc * yc * yc);
            si = mc * kr;
            sj = (MIXED ? R.mw[q] : R.mw[q] * (2.0 / 3.0)) * kr;
        }
    }
    if (a.emit) {
        const uint64_t mask = __ballot(emit);
        if (mask != 0ull) {
            const int base = __hip_atomic_load(wcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            if (emit) {
                const int pos = base + __popcll(mask & lanemask_lt());
                if (pos < WSEG) {
                    int32_t *e3 = a.stage + ((size_t)wave_g * WSEG + pos) * 3;
                    e3[0] = (int32_t)(R.ii[q] + a.o);
                    e3[1] = (int32_t)(jg + a.o);
                    e3[2] = 0;
                }
                R.kc[q] += 1;
            }
            const uint64_t act = __ballot(1);
            if ((int)__lane_id() == __ffsll((unsigned long long)act) - 1)
                __hip_atomic_store(wcnt, base + __popcll(mask), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
}

// One chunk of 64 columns against the lane's rows (binary64).  GEN = false:
// every row pairs symmetrically.  GEN = true (chunks over the group's own
// rows): mode[q] is 2 (symmetric), 1 (one-sided: the row's own chunk) or 0
// (skip), uniform over the wave.  m r^-3 as in the one-sided kick: v_rsq_f64
// (relative error below 2^-24) with its first-order correction,
// (3/2 m) y^3 (5/3 - r^2 y^2).
template <bool GEN>
__device__ __forceinline__ void sym_chunk(const SymDev &a, SymRows<false> &R,
                                          const SymCols<false> &C, int colbase, const int *mode,
                                          double &cx, double &cy, double &cz, double c53,
                                          double g2, int64_t wave_g, int *wcnt, int lane)
{
    for (int k0 = 0; k0 < 64; k0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = lane + k0 + u;
            const double2 p = C.xy[e];
            const double2 zm = C.zm[e];
#pragma unroll
            for (int q = 0; q < SYM_IPT; ++q) {
                if (GEN && mode[q] == 0) continue;
                const double dx = p.x - R.xi[q];
                const double dy = p.y - R.yi[q];
                const double dz = zm.x - R.zi[q];
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const bool cand = r2 <= g2;
                const double yv = __builtin_amdgcn_rsq(r2);
                const double y2 = yv * yv;
                const double pp = __builtin_fma(-r2, y2, c53);
                const double t = (y2 * yv) * pp;
                double si = t * zm.y;
                double sj = t * R.mw[q];
                if (cand) {
                    // the column index only here: an empty volatile asm keeps the
                    // compiler from computing it on the fast path
                    int ee = lane;
                    asm volatile("" : "+v"(ee));
                    ee += k0 + u;
                    sym_slow<false>(a, R, q, colbase + (ee & 63), r2, C.rc2[ee], C.m[ee], si, sj,
                                    wave_g, wcnt);
                }
                R.ax[q] = __builtin_fma(dx, si, R.ax[q]);
                R.ay[q] = __builtin_fma(dy, si, R.ay[q]);
                R.az[q] = __builtin_fma(dz, si, R.az[q]);
                if (!GEN || mode[q] == 2) {
                    cx = __builtin_fma(-dx, sj, cx);
                    cy = __builtin_fma(-dy, sj, cy);
                    cz = __builtin_fma(-dz, sj, cz);
                }
            }
            cx = rotate_down(cx);
            cy = rotate_down(cy);
            cz = rotate_down(cz);
        }
    }
}

// The same in mixed precision: binary32 pair arithmetic on the binary64
// differences (as the one-sided mixed kick).  A pair closer than 3 rho_ij in
// the conservative binary32 test is evaluated in binary64 (second-order
// corrected v_rsq_f64, the rare path inside rho_ij); its row term goes to the
// binary64 row sum and its column term to this wave's binary64 column sums
// nacc in LDS (at a given step the lanes hold distinct columns, and only this
// wave touches nacc, so the updates need no atomics).  The binary32 sums,
// including the sums of m / r^2 that decide the binary64 refinement of
// cancelling rows, rotate like the binary64 ones.
template <bool GEN>
__device__ __forceinline__ void sym_chunk_mixed(const SymDev &a, SymRows<true> &R,
                                                const SymCols<true> &C, double (*nacc)[64],
                                                int colbase, const int *mode, float &cx,
                                                float &cy, float &cz, float &cm, double c15,
                                                double c1875, int64_t wave_g, int *wcnt, int lane)
{
    for (int k0 = 0; k0 < 64; k0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = lane + k0 + u;
            const double2 p = C.xy[e];
            const double zc = C.z[e];
            const float2 fw = C.fw[e];
#pragma unroll
            for (int q = 0; q < SYM_IPT; ++q) {
                if (GEN && mode[q] == 0) continue;
                const bool col = !GEN || mode[q] == 2;
                const double dx = p.x - R.xi[q];
                const double dy = p.y - R.yi[q];
                const double dz = zc - R.zi[q];
                const float dxf = (float)dx, dyf = (float)dy, dzf = (float)dz;
                const float r2f = __builtin_fmaf(dzf, dzf, __builtin_fmaf(dyf, dyf, dxf * dxf));
                const bool near = r2f <= vmax_f32(R.rc2fi[q], fw.y);
                const float yv = __builtin_amdgcn_rsqf(r2f);
                const float y2 = yv * yv;
                float mti = fw.x * y2, mtj = R.mif[q] * y2;
                float si = mti * yv, sj = mtj * yv;
                if (near) {
                    si = sj = mti = mtj = 0.0f;
                    int ee = lane;
                    asm volatile("" : "+v"(ee));
                    ee += k0 + u;
                    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                    const double mc = C.m[ee], rc2c = C.rc2[ee];
                    const double y = __builtin_amdgcn_rsq(r2);
                    const double yy = y * y;
                    const double e1 = __builtin_fma(-r2, yy, 1.0);
                    const double pp = __builtin_fma(e1, c1875, c15);
                    const double t3 = yy * y;
                    const double r3 = __builtin_fma(t3 * e1, pp, t3);
                    double wi = mc * r3, wj = R.mw[q] * r3;
                    if (r2 <= vmax_f64(R.rc2i[q], rc2c))
                        sym_slow<true>(a, R, q, colbase + (ee & 63), r2, rc2c, mc, wi, wj, wave_g,
                                       wcnt);
                    R.ax[q] = __builtin_fma(dx, wi, R.ax[q]);
                    R.ay[q] = __builtin_fma(dy, wi, R.ay[q]);
                    R.az[q] = __builtin_fma(dz, wi, R.az[q]);
                    if (col) {
                        const int c = ee & 63;
                        nacc[0][c] = __builtin_fma(-dx, wj, nacc[0][c]);
                        nacc[1][c] = __builtin_fma(-dy, wj, nacc[1][c]);
                        nacc[2][c] = __builtin_fma(-dz, wj, nacc[2][c]);
                    }
                }
                R.axf[q] = __builtin_fmaf(dxf, si, R.axf[q]);
                R.ayf[q] = __builtin_fmaf(dyf, si, R.ayf[q]);
                R.azf[q] = __builtin_fmaf(dzf, si, R.azf[q]);
                R.magf[q] += mti;
                if (col) {
                    cx = __builtin_fmaf(-dxf, sj, cx);
                    cy = __builtin_fmaf(-dyf, sj, cy);
                    cz = __builtin_fmaf(-dzf, sj, cz);
                    cm += mtj;
                }
            }
            cx = rotate_down(cx);
            cy = rotate_down(cy);
            cz = rotate_down(cz);
            cm = rotate_down(cm);
        }
    }
}

// Column jg (or padding) into entries t and t + 64 of an LDS chunk.  Returns
// its rc^2 (0 for padding).
template <bool MIXED>
__device__ __forceinline__ double sym_put(SymCols<MIXED> &C, int t, bool real, double x, double y,
                                          double z, double m, double rc, double widen, double far)
{
    if (!real) {
        x = y = z = far;
        m = 0.0;
        rc = 0.0;
    }
    const double2 xy = make_double2(x, y);
    const double rc2 = rc * rc;
    C.xy[t] = xy;
    C.xy[t + 64] = xy;
    if constexpr (MIXED) {
        const float2 fw = make_float2((float)m, (float)(rc2 * widen));
        C.z[t] = z;
        C.z[t + 64] = z;
        C.fw[t] = fw;
        C.fw[t + 64] = fw;
    } else {
        const double2 zm = make_double2(z, 1.5 * m);
        C.zm[t] = zm;
        C.zm[t + 64] = zm;
    }
    C.rc2[t] = rc2;
    C.rc2[t + 64] = rc2;
    C.m[t] = m;
    C.m[t + 64] = m;
    return rc2;
}

// Column sums of chunk cc (columns cc*64 + lane) of group g: the waves' sums
// in wave order.
template <bool MIXED>
__device__ __forceinline__ void sym_colsum(const SymDev &a, const SymSmem<MIXED> &sm, int b,
                                           int64_t cc, int64_t g, int lane)
{
    constexpr int NC = MIXED ? 4 : 3;
    const SymShape &h = a.sh;
    int l = lane;   // opaque copy: the index is formed here, not kept live
    asm volatile("" : "+v"(l));
    const int j = (int)(cc * 64) + l;
    if (j >= h.n) return;
    const int64_t row0 = g * SYM_RG;
    double *cp = a.colpart + (size_t)NC * h.coloff(g) - row0 + j;
    const int64_t L = h.collen(g);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double t = sm.acc[b][c][0][lane];
#pragma unroll
        for (int v = 1; v < SYM_NW; ++v) t += sm.acc[b][c][v][lane];
        cp[c * L] = t;
    }
}

// At most 128 VGPRs (4 waves per SIMD, 4 blocks per CU); the few values this
// moves to scratch are reloaded once per chunk, not per step (unrolling 4
// steps, or 5 waves per SIMD, spill inside the step loop: 15 % slower).
// Tile (g, s) of the system described by a (its shape, and for a batch its
// arrays from its first body on), stored as tile sid.
template <bool MIXED>
__device__ __forceinline__ void sym_tile_run(const SymDev &a, int64_t g, int64_t s, int64_t sid,
                                             SymSmem<MIXED> &sm)
{
    const SymShape &h = a.sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n = h.n;
    const int64_t row0 = g * SYM_RG;
    const int64_t rowend = row0 + SYM_RG < n ? row0 + SYM_RG : n;
    const int64_t col0 = row0 + s * h.W;
    const int64_t col1 = col0 + h.W < n ? col0 + h.W : n;
    const int nch = (int)((col1 - col0 + 63) / 64);
    const int64_t wave_g = sid * SYM_NW + w;
    const bool diag = s < h.d;
    const int vzero = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
    const double c53 = a.c53 + (double)vzero;
    const double c15 = a.c15 + (double)vzero, c1875 = a.c1875 + (double)vzero;

    SymRows<MIXED> R;
    int64_t rch[SYM_IPT];   // global 64-row chunk of each row slot
#pragma unroll
    for (int q = 0; q < SYM_IPT; ++q) {
        const int cq = q * SYM_NW + w;
        const int64_t i = row0 + (int64_t)cq * 64 + lane;
        rch[q] = (row0 >> 6) + cq;
        R.ii[q] = i < rowend ? (int)i : -1;
        double mi = 0.0;
        if (i < rowend) {
            R.xi[q] = a.x[i];
            R.yi[q] = a.y[i];
            R.zi[q] = a.z[i];
            const double r = a.rc[i];
            R.rc2i[q] = r * r;
            mi = a.m[i];
        } else {
            R.xi[q] = R.yi[q] = R.zi[q] = a.far_row;
            R.rc2i[q] = 0.0;
        }
        R.mw[q] = MIXED ? mi : 1.5 * mi;
        R.ax[q] = R.ay[q] = R.az[q] = 0.0;
        R.kc[q] = 0;
        if constexpr (MIXED) {
            R.mag[q] = 0.0;
            R.rc2fi[q] = (float)(R.rc2i[q] * a.widen);
            R.mif[q] = (float)mi;
            R.axf[q] = R.ayf[q] = R.azf[q] = R.magf[q] = 0.0f;
        }
    }
    // Binary64 fast path's gate: a pair can be inside max(rc_i, rc_j) only if
    // r^2 is at most the largest rc^2 among the wave's rows and the chunk's
    // columns, so one compare against a wave-uniform bound of it (at most
    // 2^-20 above) replaces the per-pair max and compare, and the rare path
    // takes the exact test.  (The
    // mixed kernel keeps its per-pair test: the bound's registers cost it more
    // in spills than the instruction saves.)
    int rg = 0;   // high word of the bound over the wave's rows
    if constexpr (!MIXED) {
        double r2m = 0.0;
#pragma unroll
        for (int q = 0; q < SYM_IPT; ++q) r2m = vmax_f64(r2m, R.rc2i[q]);
        rg = wave_max_hi(r2m);
    }
    int *wcnt = &sm.wcnt[w];
    if (lane == 0) __hip_atomic_store(wcnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if constexpr (MIXED) {
        sm.nacc[w][0][lane] = 0.0;
        sm.nacc[w][1][lane] = 0.0;
        sm.nacc[w][2][lane] = 0.0;
    }

    // chunk 0 by wave 0
    if (w == 0) {
        const int jg = (int)col0 + lane;
        const bool real = jg < col1;
        double x = 0, y = 0, z = 0, m = 0, rc = 0;
        if (real) {
            x = a.x[jg]; y = a.y[jg]; z = a.z[jg]; m = a.m[jg]; rc = a.rc[jg];
            if (!(rc >= 0.0 && rc < INFINITY)) atomicOr(a.status, ST_RCRIT);
        }
        const double gv = sym_put<MIXED>(sm.col[0], lane, real, x, y, z, m, rc, a.widen, a.far_col);
        if constexpr (!MIXED) {
            const int gm = wave_max_hi(gv);
            if (lane == 0) sm.gmax[0] = gm;
        }
    }
    __syncthreads();

    const int64_t cc0 = col0 >> 6;
    for (int kc = 0; kc < nch; ++kc) {
        const int b = kc & 1;
        const int64_t cc = cc0 + kc;
        // column sums of the previous chunk
        if (kc > 0 && w == (kc - 1) % SYM_NW) sym_colsum<MIXED>(a, sm, b ^ 1, cc - 1, g, lane);
        // next chunk into registers (loader wave)
        const bool loader = kc + 1 < nch && w == (kc + 1) % SYM_NW;
        double px = 0, py = 0, pz = 0, pm = 0, prc = 0;
        bool preal = false;
        if (loader) {
            const int jg = (int)((cc + 1) * 64) + lane;
            preal = jg < col1;
            if (preal) {
                px = a.x[jg]; py = a.y[jg]; pz = a.z[jg]; pm = a.m[jg]; prc = a.rc[jg];
            }
        }
        const int colbase = (int)(cc * 64);
        bool full = !diag;
        int mode[SYM_IPT] = {};
        if (diag) {
            full = true;
#pragma unroll
            for (int q = 0; q < SYM_IPT; ++q) {
                mode[q] = cc > rch[q] ? 2 : (cc == rch[q] ? 1 : 0);
                full = full && mode[q] == 2;
            }
        }
        if constexpr (MIXED) {
            float cx = 0.0f, cy = 0.0f, cz = 0.0f, cm = 0.0f;
            if (full)
                sym_chunk_mixed<false>(a, R, sm.col[b], sm.nacc[w], colbase, mode, cx, cy, cz, cm,
                                       c15, c1875, wave_g, wcnt, lane);
            else
                sym_chunk_mixed<true>(a, R, sm.col[b], sm.nacc[w], colbase, mode, cx, cy, cz, cm,
                                      c15, c1875, wave_g, wcnt, lane);
            // binary32 row sums of the chunk into binary64
#pragma unroll
            for (int q = 0; q < SYM_IPT; ++q) {
                R.ax[q] += (double)R.axf[q];
                R.ay[q] += (double)R.ayf[q];
                R.az[q] += (double)R.azf[q];
                R.mag[q] += (double)R.magf[q];
                R.axf[q] = R.ayf[q] = R.azf[q] = R.magf[q] = 0.0f;
            }
            sm.acc[b][0][w][lane] = (double)cx + sm.nacc[w][0][lane];
            sm.acc[b][1][w][lane] = (double)cy + sm.nacc[w][1][lane];
            sm.acc[b][2][w][lane] = (double)cz + sm.nacc[w][2][lane];
            sm.acc[b][3][w][lane] = (double)cm;
            sm.nacc[w][0][lane] = 0.0;
            sm.nacc[w][1][lane] = 0.0;
            sm.nacc[w][2][lane] = 0.0;
        } else {
            const double g2 =
                bound_of_hi(max(rg, __builtin_amdgcn_readfirstlane(sm.gmax[b])));
            double cx = 0.0, cy = 0.0, cz = 0.0;
            if (full)
                sym_chunk<false>(a, R, sm.col[b], colbase, mode, cx, cy, cz, c53, g2, wave_g, wcnt,
                                 lane);
            else
                sym_chunk<true>(a, R, sm.col[b], colbase, mode, cx, cy, cz, c53, g2, wave_g, wcnt,
                                lane);
            sm.acc[b][0][w][lane] = cx;
            sm.acc[b][1][w][lane] = cy;
            sm.acc[b][2][w][lane] = cz;
        }
        if (loader) {
            if (preal && !(prc >= 0.0 && prc < INFINITY)) atomicOr(a.status, ST_RCRIT);
            const double gv = sym_put<MIXED>(sm.col[b ^ 1], lane, preal, px, py, pz, pm, prc,
                                              a.widen, a.far_col);
            if constexpr (!MIXED) {
                const int gm = wave_max_hi(gv);
                if (lane == 0) sm.gmax[b ^ 1] = gm;
            }
        }
        __syncthreads();
    }
    if (w == (nch - 1) % SYM_NW) sym_colsum<MIXED>(a, sm, (nch - 1) & 1, cc0 + nch - 1, g, lane);
    constexpr int NC = MIXED ? 4 : 3;
#pragma unroll
    for (int q = 0; q < SYM_IPT; ++q) {
        if (R.ii[q] < 0) continue;
        const int64_t off = R.ii[q] - row0;
        double *p = a.rowpart + (size_t)sid * NC * SYM_RG + off;
        p[0] = R.ax[q];
        p[SYM_RG] = R.ay[q];
        p[2 * SYM_RG] = R.az[q];
        if constexpr (MIXED) p[3 * SYM_RG] = R.mag[q];
        if (a.emit) a.cnt[(size_t)sid * SYM_RG + off] = R.kc[q];
    }
    if (a.emit && lane == 0)
        a.wcount[wave_g] = __hip_atomic_load(wcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

template <bool MIXED>
__global__ __launch_bounds__(SYM_NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_kick_sym(
    SymDev a)
{
    __shared__ SymSmem<MIXED> sm;
    if (MIXED && blockIdx.x == 0 && threadIdx.x == 0) *a.refine_cnt = 0;
    int64_t g, s;
    sym_tile(a.sh, blockIdx.x, g, s);
    if (s < 0) return;   // (uniform over the block)
    sym_tile_run<MIXED>(a, g, s, a.sh.tb(g) + s, sm);
}

// Batch: one block per tile, tiles launched in decreasing order of work
// (order[t] is the storage number of the t-th tile).  Binary64.
__global__ __launch_bounds__(SYM_NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_kick_sym_b(
    SymDev base, SymBatch b)
{
    __shared__ SymSmem<false> sm;
    const int64_t sid = b.order[blockIdx.x];
    const SymTileB t = b.tiles[sid];
    const SymSys ss = b.sys[t.sys];
    SymDev a = base;
    a.sh = ss.sh;
    a.o = ss.o;
    a.x += ss.o;
    a.y += ss.o;
    a.z += ss.o;
    a.m += ss.o;
    a.rc += ss.o;
    a.colpart += ss.cbase;
    sym_tile_run<false>(a, t.g, t.s, sid, sm);
}

// Place the staged pairs of the symmetric kick (one wave of 64 threads per
// kick wave).  Rank of a pair inside its (row, tile): the number of pairs of
// the same row with a smaller j in the wave's segment.  A wave whose segment
// overflowed is recomputed over its rows and the tile's columns, j ascending.
struct SymScatterDev {
    SymShape sh;                    // one system (b.tiles null)
    SymBatch b;                     // batch: tile and system descriptors
    const double *x, *y, *z, *rc;
    const int32_t *cnt, *stage, *wcount;
    const int32_t *rowloc;
    const int64_t *boff;
    int32_t *pi, *pj;
    int64_t capacity;
};

__global__ __launch_bounds__(64) void k_pairs_scatter_sym(SymScatterDev d)
{
    __shared__ int32_t si_[WSEG], sj_[WSEG];
    const int lane = threadIdx.x;
    const int64_t wave_g = blockIdx.x;
    const int64_t sid = wave_g / SYM_NW;
    const int w = (int)(wave_g % SYM_NW);
    SymShape h;
    int64_t g, s, o = 0;
    if (d.b.tiles) {
        const SymTileB t = d.b.tiles[sid];
        const SymSys ss = d.b.sys[t.sys];
        h = ss.sh;
        o = ss.o;
        g = t.g;
        s = t.s;
    } else {
        h = d.sh;
        g = sym_group_of(h, sid);
        s = sid - h.tb(g);
    }
    const int64_t row0 = g * SYM_RG;   // (local to the system)
    const int nst = d.wcount[wave_g];
    if (nst <= WSEG) {
        for (int e = lane; e < nst; e += 64) {
            const int32_t *e3 = d.stage + ((size_t)wave_g * WSEG + e) * 3;
            si_[e] = e3[0];
            sj_[e] = e3[1];
        }
        __syncthreads();
        for (int e = lane; e < nst; e += 64) {
            const int32_t i = si_[e], j = sj_[e];
            int rank = 0;
            for (int f = 0; f < nst; ++f) rank += (si_[f] == i && sj_[f] < j) ? 1 : 0;
            const int64_t pos = d.boff[i / RB] + d.rowloc[i] +
                                d.cnt[(size_t)sid * SYM_RG + (i - o - row0)] + rank;
            if (pos < d.capacity) {
                d.pi[pos] = i;
                d.pj[pos] = j;
            }
        }
        return;
    }
    const int64_t n = h.n;
    const int64_t rowend = row0 + SYM_RG < n ? row0 + SYM_RG : n;
    const int64_t col0 = row0 + s * h.W;
    const int64_t col1 = col0 + h.W < n ? col0 + h.W : n;
    for (int q = 0; q < SYM_IPT; ++q) {
        const int64_t li = row0 + (int64_t)(q * SYM_NW + w) * 64 + lane;
        if (li >= rowend) continue;
        const int64_t i = o + li;
        int64_t pos = d.boff[i / RB] + d.rowloc[i] + d.cnt[(size_t)sid * SYM_RG + (li - row0)];
        const double xi = d.x[i], yi = d.y[i], zi = d.z[i];
        const double rci = d.rc[i];
        const double rc2i = rci * rci;
        for (int64_t lj = (col0 > li + 1 ? col0 : li + 1); lj < col1; ++lj) {
            const int64_t j = o + lj;
            const double dx = d.x[j] - xi, dy = d.y[j] - yi, dz = d.z[j] - zi;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double rcj = d.rc[j];
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

static SymDev sym_dev(const SymShape &h, bool mixed, double widen, const double *x, const double *y,
                      const double *z, const double *m, const double *rc, double *rowpart,
                      double *colpart, int32_t *cnt, int32_t *stage, int32_t *wcount,
                      int32_t *status, int32_t *refine_cnt, bool emit)
{
    SymDev a;
    a.x = x; a.y = y; a.z = z; a.m = m; a.rc = rc;
    a.sh = h;
    a.rowpart = rowpart;
    a.colpart = colpart;
    a.cnt = cnt;
    a.stage = stage;
    a.wcount = wcount;
    a.status = status;
    a.refine_cnt = refine_cnt;
    a.o = 0;
    a.emit = emit ? 1 : 0;
    a.ps = mixed ? 4 : 3;
    a.c53 = 5.0 / 3.0;
    a.c15 = 1.5;
    a.c1875 = 1.875;
    a.widen = widen;
    a.far_row = SYM_FAR_ROW;
    a.far_col = SYM_FAR_COL;
    return a;
}

hipError_t launch_kick_sym(const SymShape &h, bool mixed, double widen, const double *x,
                           const double *y, const double *z, const double *m, const double *rc,
                           double *rowpart, double *colpart, int32_t *cnt, int32_t *stage,
                           int32_t *wcount, int32_t *status, int32_t *refine_cnt, bool emit,
                           hipStream_t s)
{
    const SymDev a = sym_dev(h, mixed, widen, x, y, z, m, rc, rowpart, colpart, cnt, stage,
                             wcount, status, refine_cnt, emit);
    const int64_t blocks = h.tfull + h.G * h.d;
    if (mixed)
        hipLaunchKernelGGL(k_kick_sym<true>, dim3((unsigned)blocks), dim3(SYM_NT), 0, s, a);
    else
        hipLaunchKernelGGL(k_kick_sym<false>, dim3((unsigned)blocks), dim3(SYM_NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_kick_sym_b(const SymBatch &b, const double *x, const double *y,
                             const double *z, const double *m, const double *rc, double *rowpart,
                             double *colpart, int32_t *cnt, int32_t *stage, int32_t *wcount,
                             int32_t *status, bool emit, hipStream_t s)
{
    const SymDev a = sym_dev(SymShape(), false, 0.0, x, y, z, m, rc, rowpart, colpart, cnt, stage,
                             wcount, status, nullptr, emit);
    if (b.T == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_sym_b, dim3((unsigned)b.T), dim3(SYM_NT), 0, s, a, b);
    return hipGetLastError();
}

hipError_t launch_scatter_sym(const SymShape &h, const SymBatch *b, const double *x,
                              const double *y, const double *z, const double *rc,
                              const int32_t *cnt, const int32_t *stage, const int32_t *wcount,
                              const int32_t *rowloc, const int64_t *boff, genga_pairs *pairs,
                              hipStream_t s)
{
    SymScatterDev d;
    d.sh = h;
    d.b = b ? *b : SymBatch{nullptr, nullptr, nullptr, 0, 0};
    d.x = x; d.y = y; d.z = z; d.rc = rc;
    d.cnt = cnt;
    d.stage = stage;
    d.wcount = wcount;
    d.rowloc = rowloc;
    d.boff = boff;
    d.pi = pairs->i;
    d.pj = pairs->j;
    d.capacity = pairs->capacity;
    const int64_t T = b ? b->T : h.T;
    if (T == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs_scatter_sym, dim3((unsigned)(T * SYM_NW)), dim3(64), 0, s, d);
    return hipGetLastError();
}

}  // namespace genga
