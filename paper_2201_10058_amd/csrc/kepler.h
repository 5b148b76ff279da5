// Two-body (Kepler) propagation used by the drift FG, the Keplerian part of
// H_A in GENGA II Sect. 2.  Header-only and __host__ __device__ so that the
// same solver can also be compiled for the CPU by the host-side tests.
#pragma once

#include <math.h>
#include <stdint.h>

#ifndef GENGA_HD
#define GENGA_HD __host__ __device__
#endif

namespace genga {

enum : int32_t { KEPLER_OK = 0, KEPLER_NONFINITE = 2, KEPLER_NOCONV = 8 };

// Stumpff functions C(z) = (1 - cos sqrt z) / z, S(z) = (sqrt z - sin sqrt z) / z^(3/2)
// (and their hyperbolic continuations); power series for |z| < 1.
GENGA_HD inline void stumpff(double zz, double &C, double &S)
{
    if (fabs(zz) < 1.0) {
        // C = sum (-z)^k / (2k+2)!,  S = sum (-z)^k / (2k+3)!   (k = 0..11)
        double c = 0.0, s = 0.0;
        double fc = 1.0, fs = 1.0;
        // build from the highest term down (Horner)
        double cf[12], sf[12];
        fc = 2.0;  // (2k+2)! for k = 0
        fs = 6.0;  // (2k+3)! for k = 0
        for (int k = 0; k < 12; ++k) {
            cf[k] = 1.0 / fc;
            sf[k] = 1.0 / fs;
            fc *= (double)(2 * k + 3) * (double)(2 * k + 4);
            fs *= (double)(2 * k + 4) * (double)(2 * k + 5);
        }
        for (int k = 11; k >= 0; --k) {
            c = __builtin_fma(-zz, c, cf[k]);
            s = __builtin_fma(-zz, s, sf[k]);
        }
        C = c;
        S = s;
    } else if (zz > 0.0) {
        const double sz = __builtin_sqrt(zz);
        const double h = sin(0.5 * sz);
        C = 2.0 * h * h / zz;
        S = (sz - sin(sz)) / (zz * sz);
    } else {
        const double sz = __builtin_sqrt(-zz);
        const double h = sinh(0.5 * sz);
        C = 2.0 * h * h / (-zz);
        S = (sinh(sz) - sz) / (-zz * sz);
    }
}

// Two-body propagation by the universal anomaly chi:
//   sqrt(mu) dt = sig0 chi^2 C(z) + (1 - alpha r0) chi^3 S(z) + r0 chi,  z = alpha chi^2,
//   f = 1 - chi^2 C / r0, g = dt - chi^3 S / sqrt(mu),
//   fdot = sqrt(mu) chi (z S - 1) / (r r0), gdot = 1 - chi^2 C / r.
// Newton's method kept inside a bracket (the left side increases with chi).
// Universal Kepler equation for chi (bracketed Newton):
//   sqrt(mu) dt = sig0 chi^2 C(z) + (1 - alpha r0) chi^3 S(z) + r0 chi,  z = alpha chi^2.
GENGA_HD inline int solve_chi(double r0, double sig0, double alpha, double sqmu, double dt,
                              double &chi_out)
{
    const double target = sqmu * dt;
    double chi = alpha > 0.0 ? sqmu * dt * alpha : target / r0;
    double lo = -INFINITY, hi = INFINITY;
    double C = 0.5, S = 1.0 / 6.0;
    for (int it = 0; it < 100; ++it) {
        const double zz = alpha * chi * chi;
        stumpff(zz, C, S);
        const double chi2 = chi * chi;
        const double F = sig0 * chi2 * C + (1.0 - alpha * r0) * chi2 * chi * S + r0 * chi - target;
        const double r = chi2 * C + sig0 * chi * (1.0 - zz * S) + r0 * (1.0 - zz * C);
        if (F == 0.0) {
            chi_out = chi;
            return KEPLER_OK;
        }
        if (F > 0.0) hi = chi;
        else lo = chi;
        double next = chi - F / r;
        if (!(next >= lo && next <= hi)) {
            if (lo > -INFINITY && hi < INFINITY) next = 0.5 * (lo + hi);
            else if (hi < INFINITY) next = hi - 2.0 * fabs(hi - chi) - fabs(hi) - 1.0;
            else next = lo + 2.0 * fabs(chi - lo) + fabs(lo) + 1.0;
        }
        const double step = fabs(next - chi);
        chi = next;
        if (step <= 1e-13 * fabs(chi)) {
            chi_out = chi;
            return KEPLER_OK;
        }
    }
    return KEPLER_NOCONV;
}

// Two-body propagation by the universal anomaly chi:
//   f = 1 - chi^2 C / r0, g = dt - chi^3 S / sqrt(mu),
//   fdot = sqrt(mu) chi (z S - 1) / (r r0), gdot = 1 - chi^2 C / r.
GENGA_HD inline int kepler_uv(double mu, double dt, double &x, double &y, double &z, double &vx,
                              double &vy, double &vz)
{
    const double r0 = __builtin_sqrt(x * x + y * y + z * z);
    if (!(r0 > 0.0)) return KEPLER_NONFINITE;
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double sqmu = __builtin_sqrt(mu);
    const double sig0 = (x * vx + y * vy + z * vz) / sqmu;
    const double alpha = 2.0 / r0 - v2 / mu;
    double chi;
    const int st = solve_chi(r0, sig0, alpha, sqmu, dt, chi);
    if (st != KEPLER_OK) return st;
    double C, S;
    const double zz = alpha * chi * chi;
    stumpff(zz, C, S);
    const double chi2 = chi * chi;
    const double r = chi2 * C + sig0 * chi * (1.0 - zz * S) + r0 * (1.0 - zz * C);
    const double f = 1.0 - chi2 * C / r0;
    const double g = dt - chi2 * chi * S / sqmu;
    const double fd = sqmu * chi * (zz * S - 1.0) / (r * r0);
    const double gd = 1.0 - chi2 * C / r;
    const double x0 = x, y0 = y, z0 = z;
    x = f * x0 + g * vx;
    y = f * y0 + g * vy;
    z = f * z0 + g * vz;
    vx = fd * x0 + gd * vx;
    vy = fd * y0 + gd * vy;
    vz = fd * z0 + gd * vz;
    return KEPLER_OK;
}

// Stumpff functions c_0 .. c_5 with c_n(z) = sum_k (-z)^k / (2k + n)!
// (power series for |z| < 1, closed forms and c_{n+2} = (1/n! - c_n) / z else).
GENGA_HD inline void stumpff6(double zz, double c[6])
{
    if (fabs(zz) < 1.0) {
        double f[30];
        f[0] = 1.0;
        for (int k = 1; k < 30; ++k) f[k] = f[k - 1] * (double)k;
        for (int n = 0; n < 6; ++n) {
            double acc = 0.0;
            for (int k = 11; k >= 0; --k) acc = __builtin_fma(-zz, acc, 1.0 / f[2 * k + n]);
            c[n] = acc;
        }
        return;
    }
    if (zz > 0.0) {
        const double s = __builtin_sqrt(zz);
        const double h = sin(0.5 * s);
        c[0] = cos(s);
        c[1] = sin(s) / s;
        c[2] = 2.0 * h * h / zz;
        c[3] = (s - sin(s)) / (zz * s);
    } else {
        const double s = __builtin_sqrt(-zz);
        const double h = sinh(0.5 * s);
        c[0] = cosh(s);
        c[1] = sinh(s) / s;
        c[2] = 2.0 * h * h / (-zz);
        c[3] = (sinh(s) - s) / (-zz * s);
    }
    c[4] = (0.5 - c[2]) / zz;
    c[5] = (1.0 / 6.0 - c[3]) / zz;
}

// Adjoint of kepler_uv: given the input state (X, V) and the adjoints (xb, vb)
// of the output state, overwrite xb, vb with the adjoints of the input state.
// Reverse mode through x1 = f X + g V, v1 = fdot X + gdot V with the
// universal functions U_n = chi^n c_n(alpha chi^2),
//   dU_n/dchi = U_{n-1} (dU_0/dchi = -alpha U_1),
//   dU_n/dalpha = (n U_{n+2} - chi U_{n+1}) / 2,
// and chi(alpha, r0, sig0) differentiated implicitly through the Kepler
// equation F = r0 U_1 + sig0 U_2 + U_3 - sqrt(mu) dt = 0 (dF/dchi = r).
GENGA_HD inline int kepler_uv_vjp(double mu, double dt, const double X[3], const double V[3],
                                  double xb[3], double vb[3])
{
    const double r0 = __builtin_sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    if (!(r0 > 0.0)) return KEPLER_NONFINITE;
    const double v2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    const double sqmu = __builtin_sqrt(mu);
    const double sig0 = (X[0] * V[0] + X[1] * V[1] + X[2] * V[2]) / sqmu;
    const double alpha = 2.0 / r0 - v2 / mu;
    double chi;
    const int st = solve_chi(r0, sig0, alpha, sqmu, dt, chi);
    if (st != KEPLER_OK) return st;
    double c[6];
    stumpff6(alpha * chi * chi, c);
    double U[6];
    double p = 1.0;
    for (int n = 0; n < 6; ++n) {
        U[n] = p * c[n];
        p *= chi;
    }
    const double r = r0 * U[0] + sig0 * U[1] + U[2];
    const double f = 1.0 - U[2] / r0;
    const double g = dt - U[3] / sqmu;
    const double fd = -sqmu * U[1] / (r * r0);
    const double gd = 1.0 - U[2] / r;
    double fb = 0, gb = 0, fdb = 0, gdb = 0;
    for (int k = 0; k < 3; ++k) {
        fb += xb[k] * X[k];
        gb += xb[k] * V[k];
        fdb += vb[k] * X[k];
        gdb += vb[k] * V[k];
    }
    double Xb[3], Vb[3];
    for (int k = 0; k < 3; ++k) {
        Xb[k] = f * xb[k] + fd * vb[k];
        Vb[k] = g * xb[k] + gd * vb[k];
    }
    double Ub[4] = {0.0, 0.0, 0.0, 0.0};
    double r0b = 0.0, rb = 0.0, sig0b = 0.0;
    Ub[2] += -fb / r0;
    r0b += fb * U[2] / (r0 * r0);
    Ub[3] += -gb / sqmu;
    Ub[1] += -fdb * sqmu / (r * r0);
    rb += fdb * sqmu * U[1] / (r * r * r0);
    r0b += fdb * sqmu * U[1] / (r * r0 * r0);
    Ub[2] += -gdb / r;
    rb += gdb * U[2] / (r * r);
    Ub[0] += rb * r0;
    Ub[1] += rb * sig0;
    Ub[2] += rb;
    r0b += rb * U[0];
    sig0b += rb * U[1];
    const double chib = Ub[0] * (-alpha * U[1]) + Ub[1] * U[0] + Ub[2] * U[1] + Ub[3] * U[2];
    double dUa[4];
    for (int n = 0; n < 4; ++n) dUa[n] = 0.5 * ((double)n * U[n + 2] - chi * U[n + 1]);
    double alphab = Ub[0] * dUa[0] + Ub[1] * dUa[1] + Ub[2] * dUa[2] + Ub[3] * dUa[3];
    const double Falpha = r0 * dUa[1] + sig0 * dUa[2] + dUa[3];
    const double lam = chib / r;
    alphab -= lam * Falpha;
    r0b -= lam * U[1];
    sig0b -= lam * U[2];
    r0b += alphab * (-2.0 / (r0 * r0));
    for (int k = 0; k < 3; ++k) {
        Vb[k] += alphab * (-2.0 * V[k] / mu);
        Xb[k] += sig0b * V[k] / sqmu;
        Vb[k] += sig0b * X[k] / sqmu;
        Xb[k] += r0b * X[k] / r0;
        xb[k] = Xb[k];
        vb[k] = Vb[k];
    }
    return KEPLER_OK;
}

}  // namespace genga
