/*
 * CPU oracle for the changeover-weighted kick and its companions.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference against which the HIP library is checked.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * Arithmetic is plain IEEE binary64, built with contraction disabled; the only
 * fused multiply-adds are the explicit fma() calls of the pair predicate
 * (squared separation), whose operation order is part of the predicate's
 * definition so that the encounter list has exactly one correct answer.
 *
 * Sources (GENGA II, Grimm et al. 2022):
 *   - Sect. 2, eqs. (H), (Ha), (Hb), (Hc): democratic heliocentric splitting;
 *     the kick is the interaction part H_B, HC is the Sun part H_C, the drift
 *     is the Keplerian part of H_A.
 *   - Sect. 2, eq. (rcrit): critical radius r_crit,i = max(n1 R_H,i, n2 dt v_i).
 *   - Sect. 6.2: the changeover acts for 0.1 < r/r_crit < 1 and has the form
 *     of Chambers (1999) eq. 10.
 *   - Appendix A: order of operations of one base step.
 * Readings where the paper is silent are listed at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_NONFINITE (-3)
#define OR_E_NOCONV (-6)

/* ------------------------------------------------------------------------ */
/* Changeover function (Sect. 6.2, Chambers 1999 eq. 10).                    */
/* y = (r - 0.1 rho) / (0.9 rho); K = 0 for y <= 0, 1 for y >= 1 and        */
/* y^2 / (2y^2 - 2y + 1) between.  rho = 0 gives y = +inf, i.e. K = 1.       */
/* ------------------------------------------------------------------------ */
double or_changeover_y(double y)
{
    if (!(y > 0.0)) return 0.0;
    if (y >= 1.0) return 1.0;
    return (y * y) / (2.0 * y * y - 2.0 * y + 1.0);
}

/* dK/dy on the open band, zero outside. */
double or_changeover_dy(double y)
{
    if (!(y > 0.0) || y >= 1.0) return 0.0;
    double q = 2.0 * y * y - 2.0 * y + 1.0;
    return 2.0 * y * (1.0 - y) / (q * q);
}

double or_changeover(double r, double rho)
{
    double y = (r - 0.1 * rho) / (0.9 * rho);
    if (rho == 0.0) y = INFINITY;
    return or_changeover_y(y);
}

/* ------------------------------------------------------------------------ */
/* Critical radius, eq. (rcrit).  Reading: R_H,i = |x_i| (m_i / 3 m_star)^(1/3)
 * with the heliocentric distance, and v_i = |v_i| of the democratic
 * (barycentric) velocity held in the state.                                */
/* ------------------------------------------------------------------------ */
void or_rcrit(int64_t n, const double *x, const double *y, const double *z,
              const double *vx, const double *vy, const double *vz, const double *m,
              double m_star, double dt, double n1, double n2, double *rc)
{
    for (int64_t i = 0; i < n; ++i) {
        double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
        double v = sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        double rh = r * cbrt(m[i] / (3.0 * m_star));
        double a = n1 * rh;
        double b = n2 * fabs(dt) * v;
        rc[i] = a > b ? a : b;
    }
}

/* Squared separation of the pair (i, j), the order fixed by definition:
 * d = x_j - x_i per axis, r2 = fma(dz, dz, fma(dy, dy, dx*dx)).            */
static double pair_r2(const double *x, const double *y, const double *z, int64_t i, int64_t j)
{
    double dx = x[j] - x[i];
    double dy = y[j] - y[i];
    double dz = z[j] - z[i];
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* Pair critical radius: rho_ij = max(rc_i, rc_j) (symmetric, so that the
 * weighted forces obey Newton's third law).                                 */
static double pair_rho(const double *rc, int64_t i, int64_t j)
{
    return rc[i] > rc[j] ? rc[i] : rc[j];
}

/* ------------------------------------------------------------------------ */
/* Kick accelerations (interaction part H_B, Sect. 2 and Appendix A).       */
/* a_i = G sum_{j != i} m_j K(r_ij; rho_ij) (x_j - x_i) / r_ij^3             */
/* Reading: the changeover weights the Newtonian pair force, so that K F and
 * (1 - K) F add up to F exactly (the direct solver takes the rest).          */
/* Rows [i0, i1) are evaluated; j runs in ascending order.                   */
/* precise = 0: plain binary64 sum (the timed CPU baseline).                  */
/* precise = 1: terms and sum in long double with Neumaier compensation,     */
/*              rounded once at the end (the accuracy reference).             */
/* Returns OR_E_NONFINITE if two distinct bodies coincide.                   */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Test-particle modes (Sect. 8, semi-active test particles).  Bodies       */
/* [0, nm) are massive, [nm, n) are test particles.                          */
/*   mode 0: every body acts on every other (fully interactive).             */
/*   mode 1: test particles feel the massive bodies; massive bodies feel     */
/*           only each other.                                                 */
/*   mode 2 (semi-active): as mode 1, but test particles also act on the     */
/*           massive bodies, as in the fully interactive mode.                */
/* Test particles never act on each other.  Does body j act on body i?       */
/* ------------------------------------------------------------------------ */
static int tp_acts(int mode, int64_t nm, int64_t i, int64_t j)
{
    if (mode == 0 || j < nm) return 1;
    if (i >= nm) return 0;
    return mode == 2;
}

int or_kick_acc_tp(int64_t n, const double *x, const double *y, const double *z,
                   const double *m, const double *rc, double G, int64_t nm, int mode,
                   int64_t i0, int64_t i1, int precise, double *ax, double *ay, double *az)
{
    int status = OR_OK;
    if (i0 < 0) i0 = 0;
    if (i1 > n) i1 = n;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : status)
    for (int64_t i = i0; i < i1; ++i) {
        if (!precise) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i || !tp_acts(mode, nm, i, j)) continue;
                double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                if (r2 == 0.0) { status = OR_E_NONFINITE; continue; }
                double r = sqrt(r2);
                double K = or_changeover(r, pair_rho(rc, i, j));
                double s = G * m[j] * K / (r2 * r);
                sx += s * dx; sy += s * dy; sz += s * dz;
            }
            ax[i - i0] = sx; ay[i - i0] = sy; az[i - i0] = sz;
        } else {
            long double S[3] = {0, 0, 0}, C[3] = {0, 0, 0};
            for (int64_t j = 0; j < n; ++j) {
                if (j == i || !tp_acts(mode, nm, i, j)) continue;
                long double d[3] = {(long double)x[j] - x[i], (long double)y[j] - y[i],
                                    (long double)z[j] - z[i]};
                long double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 == 0.0L) { status = OR_E_NONFINITE; continue; }
                long double r = sqrtl(r2);
                long double rho = pair_rho(rc, i, j);
                long double K;
                if (rho == 0.0L) K = 1.0L;
                else {
                    long double yy = (r - 0.1L * rho) / (0.9L * rho);
                    if (!(yy > 0.0L)) K = 0.0L;
                    else if (yy >= 1.0L) K = 1.0L;
                    else K = yy * yy / (2.0L * yy * yy - 2.0L * yy + 1.0L);
                }
                long double s = (long double)G * m[j] * K / (r2 * r);
                for (int c = 0; c < 3; ++c) {
                    long double t = s * d[c];
                    long double u = S[c] + t;
                    if (fabsl(S[c]) >= fabsl(t)) C[c] += (S[c] - u) + t;
                    else C[c] += (t - u) + S[c];
                    S[c] = u;
                }
            }
            ax[i - i0] = (double)(S[0] + C[0]);
            ay[i - i0] = (double)(S[1] + C[1]);
            az[i - i0] = (double)(S[2] + C[2]);
        }
    }
    return status;
}

int or_kick_acc(int64_t n, const double *x, const double *y, const double *z,
                const double *m, const double *rc, double G, int64_t i0, int64_t i1,
                int precise, double *ax, double *ay, double *az)
{
    return or_kick_acc_tp(n, x, y, z, m, rc, G, n, 0, i0, i1, precise, ax, ay, az);
}

/* v_i += h a_i for all bodies (plain path), in test-particle mode `mode`. */
static int kick_tp(int64_t n, const double *x, const double *y, const double *z, double *vx,
                   double *vy, double *vz, const double *m, const double *rc, double G, double h,
                   int64_t nm, int mode)
{
    double *a = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!a) return -1;
    int st = or_kick_acc_tp(n, x, y, z, m, rc, G, nm, mode, 0, n, 0, a, a + n, a + 2 * n);
    for (int64_t i = 0; i < n; ++i) {
        vx[i] += h * a[i];
        vy[i] += h * a[n + i];
        vz[i] += h * a[2 * n + i];
    }
    free(a);
    return st;
}

/* v_i += h a_i for all bodies (plain path). */
int or_kick(int64_t n, const double *x, const double *y, const double *z,
            double *vx, double *vy, double *vz, const double *m, const double *rc,
            double G, double h)
{
    return kick_tp(n, x, y, z, vx, vy, vz, m, rc, G, h, n, 0);
}

/* ------------------------------------------------------------------------ */
/* Close-encounter pairs (Sect. 2 and Appendix A: pairs closer than the     */
/* critical radius go to the direct solver; Appendix B "exact reproducible   */
/* results": the list is put in a fixed, sorted order).                      */
/* Predicate: i < j and r2 < rho*rho with r2 as in pair_r2, strict '<'.      */
/* Order: i ascending, then j ascending.  Writes at most cap pairs and       */
/* returns the true count.  Brute force over all pairs.                      */
/* ------------------------------------------------------------------------ */
/* Test-particle modes 1 and 2: only pairs with a massive first body       */
/* (i < nm) are listed; two test particles never form a pair.               */
int64_t or_pairs_tp(int64_t n, const double *x, const double *y, const double *z,
                    const double *rc, int64_t nm, int mode, int64_t cap, int32_t *pi,
                    int32_t *pj)
{
    int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    if (!cnt) return -1;
    const int64_t nrow = mode == 0 ? n : (nm < n ? nm : n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        if (i >= nrow) {
            cnt[i + 1] = 0;
            continue;
        }
        for (int64_t j = i + 1; j < n; ++j) {
            double rho = pair_rho(rc, i, j);
            if (pair_r2(x, y, z, i, j) < rho * rho) ++c;
        }
        cnt[i + 1] = c;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t total = cnt[n];
    if (pi && pj) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < nrow; ++i) {
            int64_t p = cnt[i];
            if (p >= cap || cnt[i + 1] == cnt[i]) continue;
            for (int64_t j = i + 1; j < n && p < cap; ++j) {
                double rho = pair_rho(rc, i, j);
                if (pair_r2(x, y, z, i, j) < rho * rho) {
                    pi[p] = (int32_t)i;
                    pj[p] = (int32_t)j;
                    ++p;
                }
            }
        }
    }
    free(cnt);
    return total;
}

int64_t or_pairs(int64_t n, const double *x, const double *y, const double *z,
                 const double *rc, int64_t cap, int32_t *pi, int32_t *pj)
{
    return or_pairs_tp(n, x, y, z, rc, n, 0, cap, pi, pj);
}

/* ------------------------------------------------------------------------ */
/* Sun part H_C (eq. Hc): x_i += h P / m_star, P = sum_j m_j v_j.            */
/* The momentum sum is accumulated in long double.                           */
/* ------------------------------------------------------------------------ */
/* nsum: P sums bodies [0, nsum) (test-particle mode 1: the massive ones,   */
/* since its test particles act on nothing); every body is shifted.          */
static void hc_n(int64_t n, int64_t nsum, double *x, double *y, double *z, const double *vx,
                 const double *vy, const double *vz, const double *m, double m_star, double h)
{
    long double P[3] = {0, 0, 0};
    for (int64_t j = 0; j < nsum; ++j) {
        P[0] += (long double)m[j] * vx[j];
        P[1] += (long double)m[j] * vy[j];
        P[2] += (long double)m[j] * vz[j];
    }
    double px = (double)P[0], py = (double)P[1], pz = (double)P[2];
    for (int64_t i = 0; i < n; ++i) {
        x[i] += h * px / m_star;
        y[i] += h * py / m_star;
        z[i] += h * pz / m_star;
    }
}

void or_hc(int64_t n, double *x, double *y, double *z, const double *vx,
           const double *vy, const double *vz, const double *m, double m_star, double h)
{
    hc_n(n, n, x, y, z, vx, vy, vz, m, m_star, h);
}

/* ------------------------------------------------------------------------ */
/* Keplerian drift (the Kepler part of H_A, Sect. 2): every body moves on   */
/* its two-body orbit about the star with mu = G m_star for a time dt.       */
/* Formulation: Gauss f and g functions in the eccentric-anomaly change dE   */
/* (elliptic) or the hyperbolic-anomaly change dF (hyperbolic), the classic  */
/* textbook solution of the two-body problem.  Kepler's equation in dE is    */
/* solved by Newton's method safeguarded with bisection on a bracket.        */
/* Returns OR_E_NOCONV if a solve failed, OR_E_NONFINITE for r = 0.          */
/* ------------------------------------------------------------------------ */
static int kepler_one(double mu, double dt, double *X, double *V)
{
    double r0 = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    if (!(r0 > 0.0)) return OR_E_NONFINITE;
    double v2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    double u = X[0] * V[0] + X[1] * V[1] + X[2] * V[2];   /* r0 * dr/dt */
    double alpha = 2.0 / r0 - v2 / mu;                     /* 1 / a */
    double f, g, fd, gd;
    if (dt == 0.0) return OR_OK;
    if (alpha > 0.0) {
        double a = 1.0 / alpha;
        double n = sqrt(mu * alpha * alpha * alpha);
        double ec = 1.0 - r0 * alpha;           /* e cos E0 */
        double es = u / sqrt(mu * a);           /* e sin E0 */
        double M = n * dt;
        /* F(d) = d - ec sin d + es (1 - cos d) - M, F' = 1 - ec cos d + es sin d >= 1 - e */
        double e = sqrt(ec * ec + es * es);
        double lo = M - 2.0 * e - 1e-300, hi = M + 2.0 * e + 1e-300;
        double d = M;
        int ok = 0;
        for (int it = 0; it < 200; ++it) {
            double s = sin(d), c = cos(d);
            double F = d - ec * s + es * (1.0 - c) - M;
            double Fp = 1.0 - ec * c + es * s;
            if (F > 0.0) hi = d; else lo = d;
            double dn = d - F / Fp;
            if (!(dn > lo && dn < hi)) dn = 0.5 * (lo + hi);
            double step = fabs(dn - d);
            d = dn;
            if (step <= 1e-15 * (1.0 + fabs(d))) { ok = 1; break; }
        }
        if (!ok) return OR_E_NOCONV;
        double s = sin(d), c = cos(d);
        double omc = 2.0 * sin(0.5 * d) * sin(0.5 * d);  /* 1 - cos d */
        double r = a + (r0 - a) * c + sqrt(a) * (u / sqrt(mu)) * s;
        f = 1.0 - (a / r0) * omc;
        g = dt - (d - s) / n;
        fd = -sqrt(mu * a) * s / (r * r0);
        gd = 1.0 - (a / r) * omc;
    } else if (alpha < 0.0) {
        double a = 1.0 / alpha;                  /* negative */
        double n = sqrt(mu * (-alpha) * (-alpha) * (-alpha));
        double ec = 1.0 - r0 * alpha;            /* e cosh F0 */
        double es = u / sqrt(-mu * a);           /* e sinh F0 */
        double M = n * dt;
        /* G(d) = ec sinh d + es (cosh d - 1) - d - M, increasing in d */
        double d = (M >= 0.0 ? 1.0 : -1.0) * log(1.0 + fabs(M) / (ec > 1.0 ? ec : 1.0));
        double lo = -1.0, hi = 1.0;
        while (ec * sinh(lo) + es * (cosh(lo) - 1.0) - lo - M > 0.0) lo *= 2.0;
        while (ec * sinh(hi) + es * (cosh(hi) - 1.0) - hi - M < 0.0) hi *= 2.0;
        if (!(d > lo && d < hi)) d = 0.5 * (lo + hi);
        int ok = 0;
        for (int it = 0; it < 400; ++it) {
            double sh = sinh(d), ch = cosh(d);
            double F = ec * sh + es * (ch - 1.0) - d - M;
            double Fp = ec * ch + es * sh - 1.0;
            if (F > 0.0) hi = d; else lo = d;
            double dn = d - F / Fp;
            if (!(dn > lo && dn < hi)) dn = 0.5 * (lo + hi);
            double step = fabs(dn - d);
            d = dn;
            if (step <= 1e-15 * (1.0 + fabs(d))) { ok = 1; break; }
        }
        if (!ok) return OR_E_NOCONV;
        double sh = sinh(d), ch = cosh(d);
        double chm1 = 2.0 * sinh(0.5 * d) * sinh(0.5 * d);  /* cosh d - 1 */
        double r = a + (r0 - a) * ch + sqrt(-a) * (u / sqrt(mu)) * sh;
        f = 1.0 + (a / r0) * chm1;
        g = dt - (sh - d) / n;
        fd = -sqrt(-mu * a) * sh / (r * r0);
        gd = 1.0 + (a / r) * chm1;
    } else {
        return OR_E_NOCONV;  /* exactly parabolic: not handled by this oracle */
    }
    double X1[3], V1[3];
    for (int c = 0; c < 3; ++c) {
        X1[c] = f * X[c] + g * V[c];
        V1[c] = fd * X[c] + gd * V[c];
    }
    memcpy(X, X1, sizeof X1);
    memcpy(V, V1, sizeof V1);
    return OR_OK;
}

int or_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
             double *vz, double mu, double dt)
{
    int status = OR_OK;
#pragma omp parallel for schedule(static) reduction(min : status)
    for (int64_t i = 0; i < n; ++i) {
        double X[3] = {x[i], y[i], z[i]}, V[3] = {vx[i], vy[i], vz[i]};
        int st = kepler_one(mu, dt, X, V);
        if (st != OR_OK) status = st;
        x[i] = X[0]; y[i] = X[1]; z[i] = X[2];
        vx[i] = V[0]; vy[i] = V[1]; vz[i] = V[2];
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* One base step without the direct solver (Appendix A):                    */
/*   Rcrit(dt); Kick(dt/2) [+ encounter list]; HC(dt/2); FG(dt); HC(dt/2);    */
/*   Kick(dt/2) with the same critical radii.                                 */
/* Reading: the critical radii are computed once from the state at the      */
/* start of the step and used by both half kicks; the encounter list is the  */
/* one of the first half kick.  The (1 - K) part (grouping + Bulirsch-Stoer) */
/* is not part of this step.  rc (length n) receives the radii used.         */
/* ------------------------------------------------------------------------ */
int64_t or_step_tp(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                   double *vz, const double *m, double *rc, double G, double m_star,
                   double dt, double n1, double n2, int64_t nm, int mode, int64_t cap,
                   int32_t *pi, int32_t *pj, int *status)
{
    int st = OR_OK, s2;
    const int64_t nsum = mode == 1 ? (nm < n ? nm : n) : n;
    or_rcrit(n, x, y, z, vx, vy, vz, m, m_star, dt, n1, n2, rc);
    int64_t np = or_pairs_tp(n, x, y, z, rc, nm, mode, cap, pi, pj);
    s2 = kick_tp(n, x, y, z, vx, vy, vz, m, rc, G, 0.5 * dt, nm, mode);
    if (s2 < st) st = s2;
    hc_n(n, nsum, x, y, z, vx, vy, vz, m, m_star, 0.5 * dt);
    s2 = or_drift(n, x, y, z, vx, vy, vz, G * m_star, dt);
    if (s2 < st) st = s2;
    hc_n(n, nsum, x, y, z, vx, vy, vz, m, m_star, 0.5 * dt);
    s2 = kick_tp(n, x, y, z, vx, vy, vz, m, rc, G, 0.5 * dt, nm, mode);
    if (s2 < st) st = s2;
    if (status) *status = st;
    return np;
}

int64_t or_step(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                double *vz, const double *m, double *rc, double G, double m_star,
                double dt, double n1, double n2, int64_t cap, int32_t *pi, int32_t *pj,
                int *status)
{
    return or_step_tp(n, x, y, z, vx, vy, vz, m, rc, G, m_star, dt, n1, n2, n, 0, cap, pi, pj,
                      status);
}

/* ------------------------------------------------------------------------ */
/* Symplectic levels (Sect. 6.2, higher-level changeover functions, and     */
/* Appendix A, the recursive encounter routine).  Level 0 is the base step   */
/* above.  With L > 1 levels, the bodies of the level-0 encounter list are   */
/* not drifted for dt; instead, starting from their state before the drift,  */
/* `substeps` sub-steps of dt / substeps advance them: each sub-step takes   */
/* new critical radii with the sub-step (same eq. rcrit), kicks every pair   */
/* of the upper level's list with the level weight for half a sub-step,     */
/* drifts the list's bodies, and kicks again.  The pairs of that list that   */
/* are closer than the new critical radius (at the sub-step's start) form    */
/* the next level's list, whose bodies are in turn advanced by sub-steps of  */
/* the sub-step instead of its drift, down to level L - 1.                   */
/* Level weights (l >= 1): W_l = prod_{k < l} (1 - K(r; rho_k)) K(r; rho_l); */
/* what is left, prod_{k < L} (1 - K(r; rho_k)), belongs to the direct       */
/* solver and is not integrated here (as for L = 1).                         */
/* Readings: a level's encounter list is taken at the start of each of its  */
/* sub-steps (the pre-check of its first kick, as at level 0); rho_k of an   */
/* upper level is the value of its current sub-step; no H_C term inside the  */
/* levels (the Sun kick stays at level 0).                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz;
    const double *m;
    double G, m_star, n1, n2;
    int levels, substeps;
    double *rc;        /* [levels][n]: the current critical radii of each level */
    int status;
    int direct;        /* integrate the deepest level's remainder (groups) */
    int64_t rk_steps;  /* fourth-order Runge-Kutta steps per group and interval */
    int64_t groups, group_max;   /* groups integrated, largest group */
    /* collisions (direct solver, R non-null): radii, contact tolerance as a */
    /* fraction of R_i + R_j, records (survivor, absorbed, lost energy)      */
    double *R;
    double *mw;        /* the masses, writable (mergers) */
    double coll_tol;
    int64_t ncoll, capcoll;
    int32_t *ci, *cj;
    double *cdU;
} LevelSys;

/* Weight of level l for the pair (i, j) at separation r. */
static double level_weight(const LevelSys *S, int l, int64_t i, int64_t j, double r)
{
    double w = 1.0;
    for (int k = 0; k < l; ++k) w *= 1.0 - or_changeover(r, pair_rho(S->rc + k * S->n, i, j));
    return w * or_changeover(r, pair_rho(S->rc + l * S->n, i, j));
}

/* The weight of level l (0 <= l <= L) for a pair at separation r with the  */
/* pair radii rho[0..L-1] of the levels: W_l for l < L, and for l = L the   */
/* remainder prod_{k<L} (1 - K(r; rho_k)) that no level takes.              */
double or_level_weight(double r, const double *rho, int L, int l)
{
    double w = 1.0;
    for (int k = 0; k < l && k < L; ++k) w *= 1.0 - or_changeover(r, rho[k]);
    return l < L ? w * or_changeover(r, rho[l]) : w;
}

/* v += h a over the pairs of the list with the level-l weight: each pair  */
/* acts on both of its bodies; a body's terms are added in the list order, */
/* which is its partners in ascending order.                               */
static void level_kick(LevelSys *S, int l, const int32_t *pi, const int32_t *pj, int64_t np,
                       double h)
{
    const int64_t n = S->n;
    double *a = (double *)calloc((size_t)(3 * n), sizeof(double));
    for (int64_t p = 0; p < np; ++p) {
        const int64_t i = pi[p], j = pj[p];
        const double dx = S->x[j] - S->x[i], dy = S->y[j] - S->y[i], dz = S->z[j] - S->z[i];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        if (r2 == 0.0) { S->status = OR_E_NONFINITE; continue; }
        const double r = sqrt(r2);
        const double w = level_weight(S, l, i, j, r);
        const double si = S->G * S->m[j] * w / (r2 * r);
        const double sj = S->G * S->m[i] * w / (r2 * r);
        a[i] += si * dx; a[n + i] += si * dy; a[2 * n + i] += si * dz;
        a[j] -= sj * dx; a[n + j] -= sj * dy; a[2 * n + j] -= sj * dz;
    }
    for (int64_t p = 0; p < np; ++p) {
        const int64_t b[2] = {pi[p], pj[p]};
        for (int q = 0; q < 2; ++q) {
            const int64_t k = b[q];
            if (a[k] == 0.0 && a[n + k] == 0.0 && a[2 * n + k] == 0.0) continue;
            S->vx[k] += h * a[k];
            S->vy[k] += h * a[n + k];
            S->vz[k] += h * a[2 * n + k];
            a[k] = a[n + k] = a[2 * n + k] = 0.0;   /* each body once */
        }
    }
    free(a);
}

/* Bodies of a pair list, ascending. */
static int64_t list_bodies(int64_t n, const int32_t *pi, const int32_t *pj, int64_t np,
                           int64_t *out)
{
    char *f = (char *)calloc((size_t)n, 1);
    for (int64_t p = 0; p < np; ++p) f[pi[p]] = f[pj[p]] = 1;
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (f[i]) out[k++] = i;
    free(f);
    return k;
}

static void drift_one(LevelSys *S, int64_t i, double dt)
{
    double X[3] = {S->x[i], S->y[i], S->z[i]}, V[3] = {S->vx[i], S->vy[i], S->vz[i]};
    const int st = kepler_one(S->G * S->m_star, dt, X, V);
    if (st != OR_OK) S->status = st;
    S->x[i] = X[0]; S->y[i] = X[1]; S->z[i] = X[2];
    S->vx[i] = V[0]; S->vy[i] = V[1]; S->vz[i] = V[2];
}

/* State of the listed bodies: save into / restore from buf[6 * k]. */
static void save_bodies(const LevelSys *S, const int64_t *b, int64_t k, double *buf)
{
    for (int64_t q = 0; q < k; ++q) {
        const int64_t i = b[q];
        double *o = buf + 6 * q;
        o[0] = S->x[i]; o[1] = S->y[i]; o[2] = S->z[i];
        o[3] = S->vx[i]; o[4] = S->vy[i]; o[5] = S->vz[i];
    }
}

static void restore_bodies(LevelSys *S, const int64_t *b, int64_t k, const double *buf)
{
    for (int64_t q = 0; q < k; ++q) {
        const int64_t i = b[q];
        const double *o = buf + 6 * q;
        S->x[i] = o[0]; S->y[i] = o[1]; S->z[i] = o[2];
        S->vx[i] = o[3]; S->vy[i] = o[4]; S->vz[i] = o[5];
    }
}

/* ------------------------------------------------------------------------ */
/* Close-encounter groups (Sect. 2; Appendix A "grouping"): the bodies of a */
/* pair list joined by its pairs, i.e. the connected components of the pair  */
/* graph.  label[b] = the smallest body of b's group for the list's bodies,  */
/* -1 for every other body.  Breadth-first search from each unlabelled body  */
/* in ascending order.                                                       */
/* ------------------------------------------------------------------------ */
void or_groups(int64_t n, const int32_t *pi, const int32_t *pj, int64_t np, int32_t *label)
{
    int64_t *deg = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *nbr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * np + 1));
    int64_t *fill = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t p = 0; p < np; ++p) {
        ++deg[pi[p] + 1];
        ++deg[pj[p] + 1];
    }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    for (int64_t p = 0; p < np; ++p) {
        nbr[deg[pi[p]] + fill[pi[p]]++] = pj[p];
        nbr[deg[pj[p]] + fill[pj[p]]++] = pi[p];
    }
    for (int64_t i = 0; i < n; ++i) label[i] = -1;
    for (int64_t s0 = 0; s0 < n; ++s0) {
        if (label[s0] >= 0 || deg[s0 + 1] == deg[s0]) continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = s0;
        label[s0] = (int32_t)s0;
        while (head < tail) {
            const int64_t b = queue[head++];
            for (int64_t e = deg[b]; e < deg[b + 1]; ++e) {
                const int64_t c = nbr[e];
                if (label[c] < 0) {
                    label[c] = (int32_t)s0;
                    queue[tail++] = c;
                }
            }
        }
    }
    free(deg); free(nbr); free(fill); free(queue);
}

/* ------------------------------------------------------------------------ */
/* The direct solver's share (Sect. 2, Sect. 6.1): the bodies of one group   */
/* move under the star's Kepler force and the part of their mutual forces   */
/* that no symplectic level took, R(r) = prod_{k <= l} (1 - K(r; rho_k)),   */
/* with the radii of the levels as they are (rc[k n + i]):                  */
/*   dx_i/dt = v_i,                                                         */
/*   dv_i/dt = -G m_star x_i / |x_i|^3 + G sum_{j in group} m_j R d / r^3.   */
/* This reference integrates that flow with the classical fourth-order      */
/* Runge-Kutta method in rk_steps equal steps (pinned against scipy's      */
/* DOP853 at tight tolerance).                                              */
/* ------------------------------------------------------------------------ */
static void direct_rhs(const double *m, const double *rc, int64_t n, int lmax, double G,
                       double mu, const int64_t *mem, int64_t g, const double *Y, double *F)
{
    for (int64_t a = 0; a < g; ++a) {
        const double *ya = Y + 6 * a;
        double *fa = F + 6 * a;
        fa[0] = ya[3]; fa[1] = ya[4]; fa[2] = ya[5];
        const double r2s = ya[0] * ya[0] + ya[1] * ya[1] + ya[2] * ya[2];
        const double rs = sqrt(r2s);
        double ax = -mu * ya[0] / (r2s * rs), ay = -mu * ya[1] / (r2s * rs),
               az = -mu * ya[2] / (r2s * rs);
        for (int64_t b = 0; b < g; ++b) {
            if (b == a) continue;
            const double *yb = Y + 6 * b;
            const double dx = yb[0] - ya[0], dy = yb[1] - ya[1], dz = yb[2] - ya[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double r = sqrt(r2);
            double R = 1.0;
            for (int k = 0; k <= lmax; ++k)
                R *= 1.0 - or_changeover(r, pair_rho(rc + (int64_t)k * n, mem[a], mem[b]));
            const double s = G * m[mem[b]] * R / (r2 * r);
            ax += s * dx; ay += s * dy; az += s * dz;
        }
        fa[3] = ax; fa[4] = ay; fa[5] = az;
    }
}

static void direct_rk4(const double *m, const double *rc, int64_t n, int lmax, double G,
                       double mu, const int64_t *mem, int64_t g, double *Y, double dt,
                       int64_t steps)
{
    const int64_t w = 6 * g;
    double *k1 = (double *)malloc(sizeof(double) * (size_t)(5 * w));
    double *k2 = k1 + w, *k3 = k2 + w, *k4 = k3 + w, *T = k4 + w;
    const double h = dt / (double)steps;
    for (int64_t st = 0; st < steps; ++st) {
        direct_rhs(m, rc, n, lmax, G, mu, mem, g, Y, k1);
        for (int64_t q = 0; q < w; ++q) T[q] = Y[q] + 0.5 * h * k1[q];
        direct_rhs(m, rc, n, lmax, G, mu, mem, g, T, k2);
        for (int64_t q = 0; q < w; ++q) T[q] = Y[q] + 0.5 * h * k2[q];
        direct_rhs(m, rc, n, lmax, G, mu, mem, g, T, k3);
        for (int64_t q = 0; q < w; ++q) T[q] = Y[q] + h * k3[q];
        direct_rhs(m, rc, n, lmax, G, mu, mem, g, T, k4);
        for (int64_t q = 0; q < w; ++q)
            Y[q] += h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    }
    free(k1);
}

/* ------------------------------------------------------------------------ */
/* Collisions inside the direct solver (Sect. 7, collision handling): two   */
/* members whose distance falls below R_a + R_b merge into one body.  The   */
/* fixed steps of the flow are checked after each step; the first pair found */
/* (member order) is traced back to its contact time by bisection of that   */
/* step's length, until the overlap is below coll_tol of R_a + R_b (the      */
/* paper's collision precision), and merged there:                          */
/*   x = (m_a x_a + m_b x_b)/(m_a + m_b), v likewise, m = m_a + m_b,          */
/*   R = (R_a^3 + R_b^3)^(1/3), lost energy                                  */
/*   dU = 1/2 m_a m_b/(m_a + m_b) |v_a - v_b|^2 - G m_a m_b / r_ab.            */
/* The survivor is the more massive body, or the lower index for equal      */
/* masses.  Readings: the absorbed body stays in the arrays as a massless,   */
/* sizeless ghost parked at x = (1e6 + index, 0, 0) AU at rest, far from    */
/* every other body (the caller may compact the arrays); spin is not        */
/* tracked.                                                                  */
/* ------------------------------------------------------------------------ */
static void rk4_step(const double *m, const double *rc, int64_t n, int lmax, double G, double mu,
                     const int64_t *mem, int64_t g, double *Y, double h, double *wk)
{
    const int64_t w = 6 * g;
    double *k1 = wk, *k2 = k1 + w, *k3 = k2 + w, *k4 = k3 + w, *T = k4 + w;
    direct_rhs(m, rc, n, lmax, G, mu, mem, g, Y, k1);
    for (int64_t q = 0; q < w; ++q) T[q] = Y[q] + 0.5 * h * k1[q];
    direct_rhs(m, rc, n, lmax, G, mu, mem, g, T, k2);
    for (int64_t q = 0; q < w; ++q) T[q] = Y[q] + 0.5 * h * k2[q];
    direct_rhs(m, rc, n, lmax, G, mu, mem, g, T, k3);
    for (int64_t q = 0; q < w; ++q) T[q] = Y[q] + h * k3[q];
    direct_rhs(m, rc, n, lmax, G, mu, mem, g, T, k4);
    for (int64_t q = 0; q < w; ++q) Y[q] += h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
}

static double sep(const double *Y, int64_t a, int64_t b)
{
    const double dx = Y[6 * b] - Y[6 * a], dy = Y[6 * b + 1] - Y[6 * a + 1],
                 dz = Y[6 * b + 2] - Y[6 * a + 2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* First overlapping pair (a < b in member order) of the group, or 0. */
static int find_overlap(const double *R, const int64_t *mem, int64_t g, const double *Y,
                        int64_t *pa, int64_t *pb)
{
    for (int64_t a = 0; a < g; ++a)
        for (int64_t b = a + 1; b < g; ++b) {
            const double rs = R[mem[a]] + R[mem[b]];
            if (rs > 0.0 && sep(Y, a, b) < rs) {
                *pa = a;
                *pb = b;
                return 1;
            }
        }
    return 0;
}

static void merge_members(LevelSys *S, const int64_t *mem, double *Y, int64_t a, int64_t b)
{
    const int64_t ia = mem[a], ib = mem[b];
    const double ma = S->mw[ia], mb = S->mw[ib];
    /* the survivor: the more massive body, the lower index for equal masses */
    int64_t ks = a, ka = b;
    if (mb > ma || (mb == ma && ib < ia)) {
        ks = b;
        ka = a;
    }
    const int64_t is = mem[ks], iab = mem[ka];
    double *ys = Y + 6 * ks, *yk = Y + 6 * ka;
    const double M = ma + mb;
    const double *ya = Y + 6 * a, *yb = Y + 6 * b;
    double dv2 = 0.0;
    for (int c = 3; c < 6; ++c) dv2 += (ya[c] - yb[c]) * (ya[c] - yb[c]);
    const double dU = 0.5 * ma * mb / M * dv2 - S->G * ma * mb / sep(Y, a, b);
    double merged[6];
    for (int c = 0; c < 6; ++c) merged[c] = (ma * ya[c] + mb * yb[c]) / M;
    for (int c = 0; c < 6; ++c) ys[c] = merged[c];
    yk[0] = 1e6 + (double)iab;
    yk[1] = yk[2] = yk[3] = yk[4] = yk[5] = 0.0;
    const double Rs = S->R[ia], Rb = S->R[ib];
    S->R[is] = cbrt(Rs * Rs * Rs + Rb * Rb * Rb);
    S->R[iab] = 0.0;
    S->mw[is] = M;
    S->mw[iab] = 0.0;
    if (S->ncoll < S->capcoll) {
        S->ci[S->ncoll] = (int32_t)is;
        S->cj[S->ncoll] = (int32_t)iab;
        S->cdU[S->ncoll] = dU;
    }
    ++S->ncoll;
}

/* The group's flow over dt in rk_steps equal steps, with collisions. */
static void direct_group_coll(LevelSys *S, int l, const int64_t *mem, int64_t g, double dt)
{
    const int64_t n = S->n;
    double *Y = (double *)malloc(sizeof(double) * (size_t)(6 * g + 1));
    double *Y0 = (double *)malloc(sizeof(double) * (size_t)(6 * g + 1));
    double *Yt = (double *)malloc(sizeof(double) * (size_t)(6 * g + 1));
    double *wk = (double *)malloc(sizeof(double) * (size_t)(30 * g + 1));
    for (int64_t a = 0; a < g; ++a) {
        const int64_t i = mem[a];
        double *ya = Y + 6 * a;
        ya[0] = S->x[i]; ya[1] = S->y[i]; ya[2] = S->z[i];
        ya[3] = S->vx[i]; ya[4] = S->vy[i]; ya[5] = S->vz[i];
    }
    const double mu = S->G * S->m_star;
    const double h = dt / (double)S->rk_steps;
    double t = 0.0;
    for (int64_t st = 0; st < S->rk_steps; ++st) {
        const double hs = st == S->rk_steps - 1 ? dt - t : h;
        memcpy(Y0, Y, sizeof(double) * (size_t)(6 * g));
        rk4_step(S->mw, S->rc, n, l, S->G, mu, mem, g, Y, hs, wk);
        int64_t a, b;
        if (S->R && find_overlap(S->R, mem, g, Y, &a, &b)) {
            /* contact time in (0, hs]: bisection on the step length */
            double lo = 0.0, hi = hs;
            memcpy(Yt, Y, sizeof(double) * (size_t)(6 * g));
            for (int it = 0; it < 80; ++it) {
                const double rs = S->R[mem[a]] + S->R[mem[b]];
                if ((rs - sep(Yt, a, b)) / rs < S->coll_tol) break;
                const double mid = 0.5 * (lo + hi);
                double *Yc = (double *)malloc(sizeof(double) * (size_t)(6 * g));
                memcpy(Yc, Y0, sizeof(double) * (size_t)(6 * g));
                rk4_step(S->mw, S->rc, n, l, S->G, mu, mem, g, Yc, mid, wk);
                if (sep(Yc, a, b) < rs) {
                    hi = mid;
                    memcpy(Yt, Yc, sizeof(double) * (size_t)(6 * g));
                } else {
                    lo = mid;
                }
                free(Yc);
            }
            memcpy(Y, Yt, sizeof(double) * (size_t)(6 * g));
            merge_members(S, mem, Y, a, b);
            /* the rest of this step from the contact time */
            rk4_step(S->mw, S->rc, n, l, S->G, mu, mem, g, Y, hs - hi, wk);
        }
        t += hs;
    }
    for (int64_t a = 0; a < g; ++a) {
        const int64_t i = mem[a];
        const double *ya = Y + 6 * a;
        S->x[i] = ya[0]; S->y[i] = ya[1]; S->z[i] = ya[2];
        S->vx[i] = ya[3]; S->vy[i] = ya[4]; S->vz[i] = ya[5];
    }
    free(Y); free(Y0); free(Yt); free(wk);
}

/* One group alone (for the pins): state arrays of n bodies, members mem[g], */
/* radii rc[(lmax + 1) n]; the members' state is advanced by dt in place.   */
void or_direct_group(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                     double *vz, const double *m, const double *rc, int lmax, double G,
                     double m_star, const int64_t *mem, int64_t g, double dt, int64_t steps)
{
    double *Y = (double *)malloc(sizeof(double) * (size_t)(6 * g + 1));
    for (int64_t a = 0; a < g; ++a) {
        const int64_t i = mem[a];
        double *ya = Y + 6 * a;
        ya[0] = x[i]; ya[1] = y[i]; ya[2] = z[i]; ya[3] = vx[i]; ya[4] = vy[i]; ya[5] = vz[i];
    }
    direct_rk4(m, rc, n, lmax, G, G * m_star, mem, g, Y, dt, steps);
    for (int64_t a = 0; a < g; ++a) {
        const int64_t i = mem[a];
        const double *ya = Y + 6 * a;
        x[i] = ya[0]; y[i] = ya[1]; z[i] = ya[2]; vx[i] = ya[3]; vy[i] = ya[4]; vz[i] = ya[5];
    }
    free(Y);
}

/* The groups of the list (pairs of the deepest level l) advanced over dt   */
/* from the state they had before the drift (restored by the caller).      */
static void direct_groups(LevelSys *S, int l, const int32_t *pi, const int32_t *pj, int64_t np,
                          double dt)
{
    const int64_t n = S->n;
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    or_groups(n, pi, pj, np, label);
    for (int64_t r = 0; r < n; ++r) {
        if (label[r] != r) continue;          /* r is the smallest body of its group */
        int64_t g = 0;
        for (int64_t i = r; i < n; ++i)
            if (label[i] == r) mem[g++] = i;
        ++S->groups;
        if (g > S->group_max) S->group_max = g;
        if (S->R)
            direct_group_coll(S, l, mem, g, dt);
        else
            or_direct_group(n, S->x, S->y, S->z, S->vx, S->vy, S->vz, S->m, S->rc, l, S->G,
                            S->m_star, mem, g, dt, S->rk_steps);
    }
    free(label); free(mem);
}

/* Level l >= 1: advance the bodies of the list (the encounters of level   */
/* l - 1) over substeps sub-steps of dt_l each.  counts[l] accumulates the   */
/* sizes of the lists found at level l.                                     */
static void level_advance(LevelSys *S, int l, double dt_l, const int32_t *pi, const int32_t *pj,
                          int64_t np, int64_t *counts)
{
    const int64_t n = S->n;
    int64_t *bod = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * np + 1));
    const int64_t nb = list_bodies(n, pi, pj, np, bod);
    int32_t *qi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np + 1));
    int32_t *qj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np + 1));
    int64_t *sub = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * np + 1));
    double *buf = (double *)malloc(sizeof(double) * 6 * (size_t)(2 * np + 1));
    double *rcl = S->rc + l * n;
    for (int s = 0; s < S->substeps; ++s) {
        /* critical radii of this level from the sub-step's starting state */
        for (int64_t q = 0; q < nb; ++q) {
            const int64_t i = bod[q];
            or_rcrit(1, S->x + i, S->y + i, S->z + i, S->vx + i, S->vy + i, S->vz + i, S->m + i,
                     S->m_star, dt_l, S->n1, S->n2, rcl + i);
        }
        /* this level's encounters among the list's pairs */
        int64_t nq = 0;
        for (int64_t p = 0; p < np; ++p) {
            const double rho = pair_rho(rcl, pi[p], pj[p]);
            if (pair_r2(S->x, S->y, S->z, pi[p], pj[p]) < rho * rho) {
                qi[nq] = pi[p];
                qj[nq] = pj[p];
                ++nq;
            }
        }
        counts[l] += nq;
        const int deeper = l < S->levels - 1 && nq > 0;
        const int direct = S->direct && l == S->levels - 1 && nq > 0;
        level_kick(S, l, pi, pj, np, 0.5 * dt_l);
        int64_t ns = 0;
        if (deeper || direct) {
            ns = list_bodies(n, qi, qj, nq, sub);
            save_bodies(S, sub, ns, buf);
        }
        for (int64_t q = 0; q < nb; ++q) drift_one(S, bod[q], dt_l);
        if (deeper || direct) restore_bodies(S, sub, ns, buf);
        if (deeper) level_advance(S, l + 1, dt_l / S->substeps, qi, qj, nq, counts);
        if (direct) direct_groups(S, l, qi, qj, nq, dt_l);
        level_kick(S, l, pi, pj, np, 0.5 * dt_l);
    }
    free(bod); free(qi); free(qj); free(sub); free(buf);
}

/* One base step with `levels` symplectic levels of `substeps` sub-steps    */
/* (levels = 1: or_step exactly).  rc receives the level-0 radii; counts     */
/* (length levels, may be null) the summed list sizes per level.  Returns   */
/* the level-0 pair count; the level-0 list (cap entries) goes to pi, pj.   */
/* With direct != 0 the deepest level's remainder is integrated as well:    */
/* the groups of the deepest list (level-0 list for levels = 1) advance,     */
/* instead of their drift, under the direct solver's flow (rk_steps RK4     */
/* steps per group and interval); gstats (nullable) receives the number of  */
/* groups integrated and the largest group size.                            */
/* With R non-null (radii, writable; m then writable too) the direct solver */
/* merges colliding members (see above): coll receives up to capcoll        */
/* records (survivor, absorbed, lost energy), *ncoll their true number.     */
int64_t or_step_coll(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                     double *vz, double *m, double *R, double *rc, double G, double m_star,
                     double dt, double n1, double n2, int levels, int substeps, int direct,
                     int64_t rk_steps, double coll_tol, int64_t capcoll, int32_t *ci, int32_t *cj,
                     double *cdU, int64_t *ncoll, int64_t cap, int32_t *pi, int32_t *pj,
                     int64_t *counts, int64_t *gstats, int *status);

int64_t or_step_direct(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                       double *vz, const double *m, double *rc, double G, double m_star,
                       double dt, double n1, double n2, int levels, int substeps, int direct,
                       int64_t rk_steps, int64_t cap, int32_t *pi, int32_t *pj, int64_t *counts,
                       int64_t *gstats, int *status)
{
    return or_step_coll(n, x, y, z, vx, vy, vz, (double *)m, NULL, rc, G, m_star, dt, n1, n2,
                        levels, substeps, direct, rk_steps, 0.0, 0, NULL, NULL, NULL, NULL, cap,
                        pi, pj, counts, gstats, status);
}

int64_t or_step_coll(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                     double *vz, double *m, double *R, double *rc, double G, double m_star,
                     double dt, double n1, double n2, int levels, int substeps, int direct,
                     int64_t rk_steps, double coll_tol, int64_t capcoll, int32_t *ci, int32_t *cj,
                     double *cdU, int64_t *ncoll, int64_t cap, int32_t *pi, int32_t *pj,
                     int64_t *counts, int64_t *gstats, int *status)
{
    if (levels < 1) levels = 1;
    if (substeps < 1) substeps = 1;
    LevelSys S = {n, x, y, z, vx, vy, vz, m, G, m_star, n1, n2, levels, substeps, NULL, OR_OK,
                  direct, rk_steps > 0 ? rk_steps : 1, 0, 0,
                  R, m, coll_tol, 0, capcoll, ci, cj, cdU};
    S.rc = (double *)calloc((size_t)(levels * n + 1), sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)levels, sizeof(int64_t));
    or_rcrit(n, x, y, z, vx, vy, vz, m, m_star, dt, n1, n2, S.rc);
    const int64_t np = or_pairs(n, x, y, z, S.rc, 0, NULL, NULL);
    int32_t *ei = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np + 1));
    int32_t *ej = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np + 1));
    or_pairs(n, x, y, z, S.rc, np, ei, ej);
    cnt[0] = np;
    int st = kick_tp(n, x, y, z, vx, vy, vz, m, S.rc, G, 0.5 * dt, n, 0);
    if (st < S.status) S.status = st;
    hc_n(n, n, x, y, z, vx, vy, vz, m, m_star, 0.5 * dt);
    const int deeper = (levels > 1 || direct) && np > 0;
    int64_t *bod = NULL, nb = 0;
    double *buf = NULL;
    if (deeper) {
        bod = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * np));
        nb = list_bodies(n, ei, ej, np, bod);
        buf = (double *)malloc(sizeof(double) * 6 * (size_t)nb);
        save_bodies(&S, bod, nb, buf);
    }
    st = or_drift(n, x, y, z, vx, vy, vz, G * m_star, dt);
    if (st < S.status) S.status = st;
    if (deeper) {
        restore_bodies(&S, bod, nb, buf);
        if (levels > 1) level_advance(&S, 1, dt / substeps, ei, ej, np, cnt);
        else direct_groups(&S, 0, ei, ej, np, dt);
    }
    hc_n(n, n, x, y, z, vx, vy, vz, m, m_star, 0.5 * dt);
    st = kick_tp(n, x, y, z, vx, vy, vz, m, S.rc, G, 0.5 * dt, n, 0);
    if (st < S.status) S.status = st;
    for (int64_t i = 0; i < n; ++i) rc[i] = S.rc[i];
    for (int64_t p = 0; p < np && p < cap; ++p) {
        pi[p] = ei[p];
        pj[p] = ej[p];
    }
    if (counts)
        for (int l = 0; l < levels; ++l) counts[l] = cnt[l];
    if (gstats) {
        gstats[0] = S.groups;
        gstats[1] = S.group_max;
    }
    if (ncoll) *ncoll = S.ncoll;
    if (status) *status = S.status;
    free(S.rc); free(cnt); free(ei); free(ej); free(bod); free(buf);
    return np;
}

int64_t or_step_levels(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                       double *vz, const double *m, double *rc, double G, double m_star,
                       double dt, double n1, double n2, int levels, int substeps, int64_t cap,
                       int32_t *pi, int32_t *pj, int64_t *counts, int *status)
{
    return or_step_direct(n, x, y, z, vx, vy, vz, m, rc, G, m_star, dt, n1, n2, levels, substeps,
                          0, 1, cap, pi, pj, counts, NULL, status);
}

/* ------------------------------------------------------------------------ */
/* General relativity (Sect. 3): the post-Newtonian acceleration of body i  */
/* about the star (eq. apn) with mu = G (m_star + m_i),                      */
/* eta = m_star m_i / (m_star + m_i)^2, position x_i (heliocentric) and       */
/* heliocentric velocity u_i,                                                */
/*   a = -mu / (r^2 c^2) [ -2 (2 - eta) rdot u                               */
/*        + ((1 + 3 eta) u.u - 3/2 eta rdot^2 - 2 (2 + eta) mu / r) x / r ],  */
/* rdot = u.x / r, applied over h by the implicit midpoint rule (eq.         */
/* implicit): u' = u + h a(x, (u + u') / 2), iterated from the explicit       */
/* guess until the change is below 1e-16 |u'| (at most 50 times).            */
/* Readings: u_i = v_i + P / m_star with P = sum_j m_j v_j (the star moves   */
/* at -P / m_star); afterwards the barycentric velocities are recovered with */
/* the momentum kept at zero: v'_i = u'_i - P' / m_star,                     */
/* P' = sum_j m_j u'_j / (1 + M / m_star), M = sum_j m_j.                    */
/* ------------------------------------------------------------------------ */
static void apn(double mu, double eta, double c2, const double X[3], const double U[3], double A[3])
{
    const double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    const double nx = X[0] / r, ny = X[1] / r, nz = X[2] / r;
    const double rdot = nx * U[0] + ny * U[1] + nz * U[2];
    const double u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const double coef = -mu / (r * r * c2);
    const double cu = -2.0 * (2.0 - eta) * rdot;
    const double cn = (1.0 + 3.0 * eta) * u2 - 1.5 * eta * rdot * rdot - 2.0 * (2.0 + eta) * mu / r;
    A[0] = coef * (cu * U[0] + cn * nx);
    A[1] = coef * (cu * U[1] + cn * ny);
    A[2] = coef * (cu * U[2] + cn * nz);
}

void or_gr_kick(int64_t n, const double *x, const double *y, const double *z, double *vx,
                double *vy, double *vz, const double *m, double G, double m_star, double c,
                double h)
{
    double P[3] = {0.0, 0.0, 0.0}, M = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        P[0] += m[i] * vx[i];
        P[1] += m[i] * vy[i];
        P[2] += m[i] * vz[i];
        M += m[i];
    }
    const double c2 = c * c;
    double *un = (double *)malloc(sizeof(double) * (size_t)(3 * n + 1));
    for (int64_t i = 0; i < n; ++i) {
        const double mu = G * (m_star + m[i]);
        const double eta = m_star * m[i] / ((m_star + m[i]) * (m_star + m[i]));
        const double X[3] = {x[i], y[i], z[i]};
        const double U[3] = {vx[i] + P[0] / m_star, vy[i] + P[1] / m_star, vz[i] + P[2] / m_star};
        double A[3], W[3], N[3];
        apn(mu, eta, c2, X, U, A);
        for (int k = 0; k < 3; ++k) N[k] = U[k] + h * A[k];
        for (int it = 0; it < 50; ++it) {
            for (int k = 0; k < 3; ++k) W[k] = 0.5 * (U[k] + N[k]);
            apn(mu, eta, c2, X, W, A);
            double d = 0.0, s2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double nk = U[k] + h * A[k];
                d += (nk - N[k]) * (nk - N[k]);
                s2 += nk * nk;
                N[k] = nk;
            }
            if (d <= 1e-32 * s2) break;
        }
        for (int k = 0; k < 3; ++k) un[3 * i + k] = N[k];
    }
    double Q[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) Q[k] += m[i] * un[3 * i + k];
    for (int k = 0; k < 3; ++k) Q[k] /= 1.0 + M / m_star;
    for (int64_t i = 0; i < n; ++i) {
        vx[i] = un[3 * i + 0] - Q[0] / m_star;
        vy[i] = un[3 * i + 1] - Q[1] / m_star;
        vz[i] = un[3 * i + 2] - Q[2] / m_star;
    }
    free(un);
}

/* The base step with the post-Newtonian term (c > 0): its velocity update  */
/* joins each half kick, after the first and before the second, so that the */
/* step stays symmetric:                                                    */
/*   Rcrit; Kick(dt/2); GR(dt/2); HC(dt/2); FG(dt); HC(dt/2); GR(dt/2);      */
/*   Kick(dt/2).                                                            */
int64_t or_step_gr(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                   double *vz, const double *m, double *rc, double G, double m_star, double dt,
                   double n1, double n2, double c, int64_t cap, int32_t *pi, int32_t *pj,
                   int *status)
{
    int st = OR_OK, s2;
    or_rcrit(n, x, y, z, vx, vy, vz, m, m_star, dt, n1, n2, rc);
    int64_t np = or_pairs(n, x, y, z, rc, cap, pi, pj);
    s2 = kick_tp(n, x, y, z, vx, vy, vz, m, rc, G, 0.5 * dt, n, 0);
    if (s2 < st) st = s2;
    or_gr_kick(n, x, y, z, vx, vy, vz, m, G, m_star, c, 0.5 * dt);
    hc_n(n, n, x, y, z, vx, vy, vz, m, m_star, 0.5 * dt);
    s2 = or_drift(n, x, y, z, vx, vy, vz, G * m_star, dt);
    if (s2 < st) st = s2;
    hc_n(n, n, x, y, z, vx, vy, vz, m, m_star, 0.5 * dt);
    or_gr_kick(n, x, y, z, vx, vy, vz, m, G, m_star, c, 0.5 * dt);
    s2 = kick_tp(n, x, y, z, vx, vy, vz, m, rc, G, 0.5 * dt, n, 0);
    if (s2 < st) st = s2;
    if (status) *status = st;
    return np;
}

/* ------------------------------------------------------------------------ */
/* Total energy in democratic coordinates (eqs. H, Ha, Hb, Hc):              */
/* E = sum m v^2 / 2 + |sum m v|^2 / (2 m_star) - sum G m_star m / r_i        */
/*     - sum_{i<j} G m_i m_j / r_ij  (the K-weighted parts add up to 1/r).   */
/* Long double sums.                                                         */
/* ------------------------------------------------------------------------ */
double or_energy(int64_t n, const double *x, const double *y, const double *z,
                 const double *vx, const double *vy, const double *vz, const double *m,
                 double G, double m_star)
{
    long double T = 0, P[3] = {0, 0, 0}, U = 0;
    for (int64_t i = 0; i < n; ++i) {
        T += 0.5L * m[i] * ((long double)vx[i] * vx[i] + (long double)vy[i] * vy[i] +
                            (long double)vz[i] * vz[i]);
        P[0] += (long double)m[i] * vx[i];
        P[1] += (long double)m[i] * vy[i];
        P[2] += (long double)m[i] * vz[i];
        long double r = sqrtl((long double)x[i] * x[i] + (long double)y[i] * y[i] +
                              (long double)z[i] * z[i]);
        U -= (long double)G * m_star * m[i] / r;
    }
    long double W = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : W)
    for (int64_t i = 0; i < n; ++i) {
        long double wi = 0;
        for (int64_t j = i + 1; j < n; ++j) {
            long double dx = (long double)x[j] - x[i], dy = (long double)y[j] - y[i],
                        dz = (long double)z[j] - z[i];
            wi -= (long double)G * m[i] * m[j] / sqrtl(dx * dx + dy * dy + dz * dz);
        }
        W += wi;
    }
    long double Hc = (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) / (2.0L * m_star);
    return (double)(T + Hc + U + W);
}

/* ------------------------------------------------------------------------ */
/* The changeover potential (the potential whose force is the K-weighted    */
/* Newtonian force of the kick, Sect. 2 eq. Hb with the force reading):     */
/*   Phi_K(r) = -G m_i m_j / r                          for r >= rho,        */
/*   Phi_K(r) = -G m_i m_j [1/rho + int_r^rho K(s)/s^2 ds]   for r < rho,    */
/* (K = 0 below 0.1 rho, so the integral starts at max(r, 0.1 rho)).        */
/* The integral by composite Simpson's rule on 4000 intervals.              */
/* ------------------------------------------------------------------------ */
static double k_over_s2(double s, double rho)
{
    return or_changeover(s, rho) / (s * s);
}

double or_changeover_integral(double r, double rho)
{
    if (!(r < rho)) return 0.0;
    const double a = r > 0.1 * rho ? r : 0.1 * rho;
    const int m = 4000;
    const double h = (rho - a) / m;
    double acc = k_over_s2(a, rho) + k_over_s2(rho, rho);
    for (int k = 1; k < m; ++k) acc += (k & 1 ? 4.0 : 2.0) * k_over_s2(a + k * h, rho);
    return acc * h / 3.0;
}

/* E_K: the energy with the changeover potential in place of the Newtonian  */
/* pair potential for the pairs inside rho_ij (the quantity that the step   */
/* map without the direct solver conserves for fixed critical radii):       */
/*   E_K = E + sum_{i<j, r_ij < rho_ij} [Phi_K(r_ij) + G m_i m_j / r_ij].     */
/* All pairs are examined; long double sums.                                */
double or_energy_k(int64_t n, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz, const double *m,
                   const double *rc, double G, double m_star)
{
    const double E = or_energy(n, x, y, z, vx, vy, vz, m, G, m_star);
    long double corr = 0.0L;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : corr)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            const double rho = pair_rho(rc, i, j);
            const double r2 = pair_r2(x, y, z, i, j);
            if (!(r2 < rho * rho)) continue;
            const double r = sqrt(r2);
            const long double gmm = (long double)G * m[i] * m[j];
            /* Phi_K + G m m / r = G m m [1/r - 1/rho - integral] */
            corr += gmm * (1.0L / r - 1.0L / rho - (long double)or_changeover_integral(r, rho));
        }
    }
    return (double)((long double)E + corr);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
