// Symmetric adjoint of the kick: each unordered pair evaluated once and its
// terms applied to both bodies.
//
// The kick of GENGA II Sect. 2 (eq. Hb, changeover of Sect. 6.2),
//   a_k = G sum_{j != k} m_j w_kj d_kj,  d_kj = x_j - x_k,  w = K(y) / r^3,
// has, for a cotangent abar, the vector-Jacobian product
//   xbar_k  = G sum_j X_kj,  X_kj = w u + (w_r / r)(d.u) d,  u = m_k abar_j - m_j abar_k,
//   mbar_k  = -G sum_j w d.abar_j,
//   rcbar_k = G sum_{j: k owns rho_kj} K'(y) / (0.9 rho^2 r^2) d.u
// (w_r / r = K' / (0.9 rho r^4) - 3 K / r^5; "k owns rho" means rc_k > rc_j, or
// rc_k = rc_j and k < j).  With d_jk = -d and u_jk = -u, the pair gives body j
// X_jk = -X_kj, the mbar term +G w d.abar_k and the same rcbar term, so a pair
// is evaluated once for both bodies, as in the symmetric kick: rows in groups
// of 512 (4 waves, 2 rows per lane), column chunks of 64 staged in LDS, each
// lane on column (l + k) mod 64 at step k, the column sums (three X
// components and the mbar term) carried across the wave by DPP rotations;
// the rcbar terms of band pairs owned by a column go to a wave-private LDS
// sum (at a step the lanes hold distinct columns).  Chunks over the group's
// own rows are done symmetrically after the row's chunk, one-sided on it and
// not before it.
//
// Units: the staged cotangents are abar' = 3/2 scale abar, so that with
// u' = m_k abar'_j - m_j abar'_k = 3/2 u and du' = d.u' = 3/2 d.u the fast
// path (K = 1) needs, from y = v_rsq_f64(r2) and t = r2 y^2 (first order in
// e = 1 - t, as in the kick),
//   w = y^3 (5/3 - t)        = r^-3 / (3/2)  -> w u' = r^-3 u,
//   c = y^5 (5 t - 7)        = -3 r^-5 / (3/2) -> c du' d = -3 r^-5 (d.u) d,
// so X = w u' + c du' d exactly, and w d.abar'_j = r^-3 d.abar_j.  Per tile
// and row (group and column) five sums are written: X (3), sum w d.abar'
// (mbar = -G times it; columns store the negative of their +G term) and the
// rcbar sum; k_vjp_sym_reduce adds a row's tile sums in slice order, then its
// column sums in group order (no atomics, the same bits on every run).
#include "genga_internal.h"
#include <algorithm>

#include "device_common.h"
#include "sym_common.h"

namespace genga {

constexpr int VS_NC = 5;   // sums per row and column: X (3), mbar term, rcbar

struct VsymDev {
    const double *x, *y, *z, *m, *rc;
    const double *abx, *aby, *abz;
    double abscale;      // abar' = abscale * abar (3/2 scale)
    SymShape sh;
    double *rowpart;     // [T][VS_NC][SYM_RG]
    double *colpart;     // group g: [VS_NC][collen(g)] from VS_NC coloff(g)
    int32_t *status;
    double far_row, far_col;
    double c53;          // 5/3
};

struct VsymCols {        // one chunk of 64 columns, stored twice (no wrap)
    double4 xyzm[128];   // x, y, z, m
    double4 ab[128];     // abar' (3), rc^2
    double rc[128];
};

struct VsymSmem {
    VsymCols col;
    double acc[4][SYM_NW][64];   // a chunk's column sums per wave: X (3), mbar term
    double rbc[SYM_NW][64];      // rcbar of band pairs owned by the column, per wave
    double rcr[SYM_IPT][SYM_NW][64];   // the rows' critical radii (rare path)
    double rbr[SYM_IPT][SYM_NW][64];   // the rows' rcbar sums (rare path)
    int gmax;                    // high word of a bound of the chunk's largest rc^2
};

struct VsymRows {
    double xi[SYM_IPT], yi[SYM_IPT], zi[SYM_IPT], mi[SYM_IPT];
    double ax[SYM_IPT], ay[SYM_IPT], az[SYM_IPT];   // abar' of the row
    double X[SYM_IPT], Y[SYM_IPT], Z[SYM_IPT], Mb[SYM_IPT];
    int ii[SYM_IPT];   // row index, -1 for padding
    double *rcr[SYM_IPT], *rbr[SYM_IPT];   // the lane's entries of the rows' LDS values
};

// Rare path: r2 at most the wave's gate bound.  The self pair and coincident
// bodies contribute nothing (the latter set NONFINITE); inside rho_ij the
// changeover weights replace the fast w and c and the rcbar term goes to
// the owner (the row, or when col is set, the column's LDS sum); between
// rho_ij and the bound the fast weights stand.
__device__ __forceinline__ void vsym_slow(const VsymDev &a, VsymRows &R, int q, int jg, double r2,
                                          double rcj, double du, bool col, double *rbc, int c64,
                                          double &w, double &c)
{
    if (jg == R.ii[q]) {
        w = 0.0;
        c = 0.0;
        return;
    }
    if (r2 == 0.0) {
        atomicOr(a.status, ST_NONFINITE);
        w = 0.0;
        c = 0.0;
        return;
    }
    const double rck = *R.rcr[q];
    const double rho = rck > rcj ? rck : rcj;
    if (!(r2 < rho * rho)) return;
    const double yc = rsq_nr(r2);
    const double yc2 = yc * yc, yc3 = yc2 * yc;
    const double irho = rsq_nr(rho * rho);
    double K, Kp;
    changeover_kdk_of_y(__builtin_fma((r2 * yc) * irho, 1.0 / 0.9, -1.0 / 9.0), K, Kp);
    w = (K * yc3) * (2.0 / 3.0);
    const double wr_r = (Kp * (irho * (1.0 / 0.9))) * (yc2 * yc2) - (3.0 * K) * (yc3 * yc2);
    c = wr_r * (2.0 / 3.0);
    if (Kp != 0.0) {
        const double rb = ((Kp * (irho * irho)) * (1.0 / 0.9)) * yc2 * (du * (2.0 / 3.0));
        const bool row_owns = rck > rcj || (rck == rcj && R.ii[q] < jg);
        if (row_owns) *R.rbr[q] += rb;
        else if (col) rbc[c64] += rb;
    }
}

// One chunk of 64 columns against the lane's rows.  GEN = false: every row
// pairs symmetrically; GEN = true: mode[q] is 2 (symmetric), 1 (one-sided)
// or 0 (skip), uniform over the wave.
template <bool GEN>
__device__ __forceinline__ void vsym_chunk(const VsymDev &a, VsymRows &R, const VsymCols &C,
                                           int colbase, const int *mode, double &cx, double &cy,
                                           double &cz, double &cm, double *rbc, double c53,
                                           double g2, int lane)
{
    for (int k0 = 0; k0 < 64; k0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = lane + k0 + u;
            const double4 p = C.xyzm[e];
            const double4 ab = C.ab[e];
#pragma unroll
            for (int q = 0; q < SYM_IPT; ++q) {
                if (GEN && mode[q] == 0) continue;
                const bool col = !GEN || mode[q] == 2;
                const double dx = p.x - R.xi[q];
                const double dy = p.y - R.yi[q];
                const double dz = p.z - R.zi[q];
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const bool cand = r2 <= g2;
                const double yv = __builtin_amdgcn_rsq(r2);
                const double y2 = yv * yv;
                const double t = r2 * y2;
                const double y3 = y2 * yv;
                double w = y3 * (c53 - t);
                double c = (y3 * y2) * __builtin_fma(t, 5.0, -7.0);
                const double da = __builtin_fma(dz, ab.z, __builtin_fma(dy, ab.y, dx * ab.x));
                const double db =
                    __builtin_fma(dz, R.az[q], __builtin_fma(dy, R.ay[q], dx * R.ax[q]));
                const double du = __builtin_fma(R.mi[q], da, -(p.w * db));
                if (cand) {
                    // the column index only here (kept off the fast path)
                    int ee = lane;
                    asm volatile("" : "+v"(ee));
                    ee += k0 + u;
                    vsym_slow(a, R, q, colbase + (ee & 63), r2, C.rc[ee], du, col, rbc, ee & 63,
                              w, c);
                }
                const double cd = c * du;
                // X = w u' + cd d, u' = m_k abar'_j - m_j abar'_k
                const double Xx = __builtin_fma(w, __builtin_fma(R.mi[q], ab.x, -(p.w * R.ax[q])),
                                                cd * dx);
                const double Xy = __builtin_fma(w, __builtin_fma(R.mi[q], ab.y, -(p.w * R.ay[q])),
                                                cd * dy);
                const double Xz = __builtin_fma(w, __builtin_fma(R.mi[q], ab.z, -(p.w * R.az[q])),
                                                cd * dz);
                R.X[q] += Xx;
                R.Y[q] += Xy;
                R.Z[q] += Xz;
                R.Mb[q] = __builtin_fma(w, da, R.Mb[q]);
                if (col) {
                    cx -= Xx;
                    cy -= Xy;
                    cz -= Xz;
                    cm = __builtin_fma(-w, db, cm);
                }
            }
            cx = rotate_down(cx);
            cy = rotate_down(cy);
            cz = rotate_down(cz);
            cm = rotate_down(cm);
        }
    }
}

// Column j (or padding) into entries t and t + 64 of the chunk; its rc^2.
__device__ __forceinline__ double vsym_put(const VsymDev &a, VsymCols &C, int t, int j, bool real)
{
    double x = a.far_col, y = a.far_col, z = a.far_col, m = 0.0, rc = 0.0;
    double abx = 0.0, aby = 0.0, abz = 0.0;
    if (real) {
        x = a.x[j]; y = a.y[j]; z = a.z[j]; m = a.m[j]; rc = a.rc[j];
        abx = a.abscale * a.abx[j];
        aby = a.abscale * a.aby[j];
        abz = a.abscale * a.abz[j];
        if (!(rc >= 0.0 && rc < INFINITY)) atomicOr(a.status, ST_RCRIT);
    }
    const double rc2 = rc * rc;
    const double4 p = make_double4(x, y, z, m), ab = make_double4(abx, aby, abz, rc2);
    C.xyzm[t] = p;
    C.xyzm[t + 64] = p;
    C.ab[t] = ab;
    C.ab[t + 64] = ab;
    C.rc[t] = rc;
    C.rc[t + 64] = rc;
    return rc2;
}

__global__ __launch_bounds__(SYM_NT) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_kick_vjp_sym(
    VsymDev a)
{
    __shared__ VsymSmem sm;
    int64_t g, s;
    sym_tile(a.sh, blockIdx.x, g, s);
    if (s < 0) return;   // (uniform over the block)
    const SymShape &h = a.sh;
    const int64_t sid = h.tb(g) + s;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n = h.n;
    const int64_t row0 = g * SYM_RG;
    const int64_t rowend = row0 + SYM_RG < n ? row0 + SYM_RG : n;
    const int64_t col0 = row0 + s * h.W;
    const int64_t col1 = col0 + h.W < n ? col0 + h.W : n;
    const int nch = (int)((col1 - col0 + 63) / 64);
    const bool diag = s < h.d;
    const int vzero = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
    const double c53 = a.c53 + (double)vzero;

    VsymRows R;
    int64_t rch[SYM_IPT];
    double r2m = 0.0;
#pragma unroll
    for (int q = 0; q < SYM_IPT; ++q) {
        const int cq = q * SYM_NW + w;
        const int64_t i = row0 + (int64_t)cq * 64 + lane;
        rch[q] = (row0 >> 6) + cq;
        R.ii[q] = i < rowend ? (int)i : -1;
        R.rcr[q] = &sm.rcr[q][w][lane];
        R.rbr[q] = &sm.rbr[q][w][lane];
        double rci = 0.0;
        if (i < rowend) {
            R.xi[q] = a.x[i];
            R.yi[q] = a.y[i];
            R.zi[q] = a.z[i];
            R.mi[q] = a.m[i];
            rci = a.rc[i];
            R.ax[q] = a.abscale * a.abx[i];
            R.ay[q] = a.abscale * a.aby[i];
            R.az[q] = a.abscale * a.abz[i];
        } else {
            R.xi[q] = R.yi[q] = R.zi[q] = a.far_row;
            R.mi[q] = 0.0;
            R.ax[q] = R.ay[q] = R.az[q] = 0.0;
        }
        R.X[q] = R.Y[q] = R.Z[q] = R.Mb[q] = 0.0;
        *R.rcr[q] = rci;
        *R.rbr[q] = 0.0;
        r2m = vmax_f64(r2m, rci * rci);
    }
    const int rg = wave_max_hi(r2m);

    // chunk 0 by wave 0
    if (w == 0) {
        const int j = (int)col0 + lane;
        const double gv = vsym_put(a, sm.col, lane, j, j < col1);
        const int gm = wave_max_hi(gv);
        if (lane == 0) sm.gmax = gm;
    }
    __syncthreads();

    const int64_t cc0 = col0 >> 6;
    for (int kc = 0; kc < nch; ++kc) {
        const int64_t cc = cc0 + kc;
        const bool loader = kc + 1 < nch && w == (kc + 1) % SYM_NW;
        // the next chunk into registers while this one is computed
        const int jn = (int)((cc + 1) * 64) + lane;
        const bool nreal = loader && jn < col1;
        double px = 0, py = 0, pz = 0, pm = 0, prc = 0, pax = 0, pay = 0, paz = 0;
        if (nreal) {
            px = a.x[jn]; py = a.y[jn]; pz = a.z[jn]; pm = a.m[jn]; prc = a.rc[jn];
            pax = a.abx[jn]; pay = a.aby[jn]; paz = a.abz[jn];
        }
        sm.rbc[w][lane] = 0.0;
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
        const double g2 = bound_of_hi(max(rg, __builtin_amdgcn_readfirstlane(sm.gmax)));
        double cx = 0.0, cy = 0.0, cz = 0.0, cm = 0.0;
        if (full)
            vsym_chunk<false>(a, R, sm.col, colbase, mode, cx, cy, cz, cm, sm.rbc[w], c53, g2, lane);
        else
            vsym_chunk<true>(a, R, sm.col, colbase, mode, cx, cy, cz, cm, sm.rbc[w], c53, g2, lane);
        sm.acc[0][w][lane] = cx;
        sm.acc[1][w][lane] = cy;
        sm.acc[2][w][lane] = cz;
        sm.acc[3][w][lane] = cm;
        __syncthreads();
        // column sums of this chunk (waves in order), by one wave
        if (w == kc % SYM_NW) {
            int l = lane;   // opaque copy: the index is formed here, not kept live
            asm volatile("" : "+v"(l));
            const int j = (int)(cc * 64) + l;
            if (j < n) {
                double *cp = a.colpart + (size_t)VS_NC * h.coloff(g) - row0 + j;
                const int64_t L = h.collen(g);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double t = sm.acc[c][0][l];
#pragma unroll
                    for (int v = 1; v < SYM_NW; ++v) t += sm.acc[c][v][l];
                    cp[c * L] = t;
                }
                double t = sm.rbc[0][l];
#pragma unroll
                for (int v = 1; v < SYM_NW; ++v) t += sm.rbc[v][l];
                cp[4 * L] = t;
            }
        }
        if (loader) {
            if (nreal && !(prc >= 0.0 && prc < INFINITY)) atomicOr(a.status, ST_RCRIT);
            const double sc = a.abscale;
            const double4 p = nreal ? make_double4(px, py, pz, pm)
                                    : make_double4(a.far_col, a.far_col, a.far_col, 0.0);
            const double rc2 = prc * prc;
            const double4 ab = make_double4(sc * pax, sc * pay, sc * paz, rc2);
            sm.col.xyzm[lane] = p;
            sm.col.xyzm[lane + 64] = p;
            sm.col.ab[lane] = ab;
            sm.col.ab[lane + 64] = ab;
            sm.col.rc[lane] = prc;
            sm.col.rc[lane + 64] = prc;
            const int gm = wave_max_hi(rc2);
            if (lane == 0) sm.gmax = gm;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < SYM_IPT; ++q) {
        if (R.ii[q] < 0) continue;
        const int64_t off = R.ii[q] - row0;
        double *p = a.rowpart + (size_t)sid * VS_NC * SYM_RG + off;
        p[0] = R.X[q];
        p[SYM_RG] = R.Y[q];
        p[2 * SYM_RG] = R.Z[q];
        p[3 * SYM_RG] = R.Mb[q];
        p[4 * SYM_RG] = *R.rbr[q];
    }
}

// Totals per row: its tile sums in slice order, then the column sums of
// groups 0..g(i) in group order; xbar += G X, mbar -= G (mbar term), rcbar
// += G (rcbar sum).
__global__ __launch_bounds__(RB) void k_vjp_sym_reduce(const double *rowpart,
                                                       const double *colpart, SymShape h, double G,
                                                       double *xb, double *yb, double *zb,
                                                       double *mb, double *rcb)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= h.n) return;
    const int64_t grp = i / SYM_RG;
    const int64_t nsl = h.ns(grp);
    const double *rp = rowpart + (size_t)h.tb(grp) * VS_NC * SYM_RG + (i - grp * SYM_RG);
    double acc[VS_NC] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t q = 0;
    for (; q + 4 <= nsl; q += 4) {
        double v[4][VS_NC];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < VS_NC; ++c) v[k][c] = rp[(size_t)(q + k) * VS_NC * SYM_RG + c * SYM_RG];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < VS_NC; ++c) acc[c] += v[k][c];
    }
    for (; q < nsl; ++q)
#pragma unroll
        for (int c = 0; c < VS_NC; ++c) acc[c] += rp[(size_t)q * VS_NC * SYM_RG + c * SYM_RG];
    int64_t gg = 0;
    for (; gg + 4 <= grp + 1; gg += 4) {
        double v[4][VS_NC];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double *cp = colpart + (size_t)VS_NC * h.coloff(gg + k) + (i - (gg + k) * SYM_RG);
            const int64_t L = h.collen(gg + k);
#pragma unroll
            for (int c = 0; c < VS_NC; ++c) v[k][c] = cp[c * L];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < VS_NC; ++c) acc[c] += v[k][c];
    }
    for (; gg <= grp; ++gg) {
        const double *cp = colpart + (size_t)VS_NC * h.coloff(gg) + (i - gg * SYM_RG);
        const int64_t L = h.collen(gg);
#pragma unroll
        for (int c = 0; c < VS_NC; ++c) acc[c] += cp[c * L];
    }
    xb[i] += G * acc[0];
    yb[i] += G * acc[1];
    zb[i] += G * acc[2];
    mb[i] -= G * acc[3];
    rcb[i] += G * acc[4];
}

hipError_t launch_kick_vjp_sym(const SymShape &h, const genga_bodies *b, double G, double scale,
                               const double *abx, const double *aby, const double *abz,
                               genga_adjoint *adj, double *part, int32_t *status, hipStream_t s)
{
    VsymDev a;
    a.x = b->x; a.y = b->y; a.z = b->z; a.m = b->m; a.rc = b->rc;
    a.abx = abx; a.aby = aby; a.abz = abz;
    a.abscale = 1.5 * scale;
    a.sh = h;
    a.rowpart = part;
    a.colpart = part + (size_t)VS_NC * h.T * SYM_RG;
    a.status = status;
    a.far_row = 1e18;
    a.far_col = -1e18;
    a.c53 = 5.0 / 3.0;
    const int64_t blocks = h.tfull + h.G * h.d;
    hipLaunchKernelGGL(k_kick_vjp_sym, dim3((unsigned)blocks), dim3(SYM_NT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vjp_sym_reduce, dim3((unsigned)((h.n + RB - 1) / RB)), dim3(RB), 0, s,
                       (const double *)a.rowpart, (const double *)a.colpart, h, G, adj->x, adj->y,
                       adj->z, adj->m, adj->rc);
    return hipGetLastError();
}

}  // namespace genga
