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
GENGA_HD inline int kepler_uv(double mu, double dt, double &x, double &y, double &z, double &vx,
                         double &vy, double &vz)
{
    const double r0 = __builtin_sqrt(x * x + y * y + z * z);
    if (!(r0 > 0.0)) return KEPLER_NONFINITE;
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double sqmu = __builtin_sqrt(mu);
    const double sig0 = (x * vx + y * vy + z * vz) / sqmu;
    const double alpha = 2.0 / r0 - v2 / mu;
    const double target = sqmu * dt;
    double chi = alpha > 0.0 ? sqmu * dt * alpha : target / r0;
    double lo = -INFINITY, hi = INFINITY;
    double C = 0.5, S = 1.0 / 6.0, r = r0;
    bool ok = false;
    for (int it = 0; it < 100; ++it) {
        const double zz = alpha * chi * chi;
        stumpff(zz, C, S);
        const double chi2 = chi * chi;
        const double F = sig0 * chi2 * C + (1.0 - alpha * r0) * chi2 * chi * S + r0 * chi - target;
        r = chi2 * C + sig0 * chi * (1.0 - zz * S) + r0 * (1.0 - zz * C);
        if (F == 0.0) {
            ok = true;
            break;
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
            ok = true;
            break;
        }
    }
    if (!ok) return KEPLER_NOCONV;
    const double zz = alpha * chi * chi;
    stumpff(zz, C, S);
    const double chi2 = chi * chi;
    r = chi2 * C + sig0 * chi * (1.0 - zz * S) + r0 * (1.0 - zz * C);
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

}  // namespace genga
