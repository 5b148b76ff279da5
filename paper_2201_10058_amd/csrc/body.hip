// O(N) operators of the base step: critical radii (eq. rcrit), HC (eq. Hc)
// and the Keplerian drift FG (Kepler part of eq. Ha), GENGA II Sect. 2 and
// Appendix A.  One thread per body; reductions run in a fixed order.
#include "genga_internal.h"
#include "kepler.h"

namespace genga {

static_assert(KEPLER_NONFINITE == ST_NONFINITE && KEPLER_NOCONV == ST_NOCONV,
              "Kepler codes are status bits");

__global__ void k_clear_status(int32_t *status) { *status = 0; }

// r_crit,i = max(n1 R_H,i, n2 |dt| |v_i|), R_H,i = |x_i| (m_i / 3 m_star)^(1/3)
__global__ __launch_bounds__(RB) void k_rcrit(const double *x, const double *y, const double *z,
                                              const double *vx, const double *vy, const double *vz,
                                              const double *m, double *rc, int64_t n, double m_star,
                                              double dt, double n1, double n2, int32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    const double r = __builtin_sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
    const double v = __builtin_sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    const double rh = r * cbrt(m[i] / (3.0 * m_star));
    const double a = n1 * rh;
    const double b = n2 * fabs(dt) * v;
    const double out = a > b ? a : b;
    if (!(out >= 0.0 && out < INFINITY)) atomicOr(status, ST_RCRIT);
    rc[i] = out;
}

// Per-block momentum partials P_b = sum_{j in block} m_j v_j (fixed tree order).
__global__ __launch_bounds__(RB) void k_momentum_partial(const double *vx, const double *vy,
                                                         const double *vz, const double *m,
                                                         int64_t n, double *hc)
{
    __shared__ double sm[3][RB];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * RB + t;
    const double mi = i < n ? m[i] : 0.0;
    sm[0][t] = i < n ? mi * vx[i] : 0.0;
    sm[1][t] = i < n ? mi * vy[i] : 0.0;
    sm[2][t] = i < n ? mi * vz[i] : 0.0;
    __syncthreads();
    for (int h = RB / 2; h > 0; h >>= 1) {
        if (t < h) {
            sm[0][t] += sm[0][t + h];
            sm[1][t] += sm[1][t + h];
            sm[2][t] += sm[2][t + h];
        }
        __syncthreads();
    }
    if (t < 3) hc[(size_t)blockIdx.x * 3 + t] = sm[t][0];
}

// x_i += h P / m_star; every block reduces the partials in the same order.
__global__ __launch_bounds__(RB) void k_hc_apply(double *x, double *y, double *z, int64_t n,
                                                 const double *hc, int64_t nb, double h,
                                                 double m_star)
{
    __shared__ double sm[3][RB];
    const int t = threadIdx.x;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int64_t b = t; b < nb; b += RB) {
        p0 += hc[b * 3 + 0];
        p1 += hc[b * 3 + 1];
        p2 += hc[b * 3 + 2];
    }
    sm[0][t] = p0;
    sm[1][t] = p1;
    sm[2][t] = p2;
    __syncthreads();
    for (int hh = RB / 2; hh > 0; hh >>= 1) {
        if (t < hh) {
            sm[0][t] += sm[0][t + hh];
            sm[1][t] += sm[1][t + hh];
            sm[2][t] += sm[2][t + hh];
        }
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * RB + t;
    if (i >= n) return;
    x[i] += (h * sm[0][0]) / m_star;
    y[i] += (h * sm[1][0]) / m_star;
    z[i] += (h * sm[2][0]) / m_star;
}

__global__ __launch_bounds__(RB) void k_drift(double *x, double *y, double *z, double *vx,
                                              double *vy, double *vz, int64_t n, double mu,
                                              double dt, int32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    double X = x[i], Y = y[i], Z = z[i], VX = vx[i], VY = vy[i], VZ = vz[i];
    const int st = kepler_uv(mu, dt, X, Y, Z, VX, VY, VZ);
    if (st) atomicOr(status, st);
    x[i] = X; y[i] = Y; z[i] = Z;
    vx[i] = VX; vy[i] = VY; vz[i] = VZ;
}

// ---------------------------------------------------------------------------
// Batched systems: body i belongs to system sysid[i]; per-system m_star, dt,
// n1, n2 arrays.  hfac scales each system's dt (0.5 for a half step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_rcrit_b(const double *x, const double *y, const double *z,
                                                const double *vx, const double *vy,
                                                const double *vz, const double *m, double *rc,
                                                int64_t n, const int32_t *sysid,
                                                const double *m_star, const double *dt,
                                                const double *n1, const double *n2,
                                                int32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    const int s = sysid[i];
    const double r = __builtin_sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
    const double v = __builtin_sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    const double rh = r * cbrt(m[i] / (3.0 * m_star[s]));
    const double a = n1[s] * rh;
    const double b = n2[s] * fabs(dt[s]) * v;
    const double out = a > b ? a : b;
    if (!(out >= 0.0 && out < INFINITY)) atomicOr(status, ST_RCRIT);
    rc[i] = out;
}

// P_s = sum over the bodies of system s of m v; one block per system, fixed order.
__global__ __launch_bounds__(RB) void k_momentum_sys(const double *vx, const double *vy,
                                                     const double *vz, const double *m,
                                                     const int64_t *offsets, double *P)
{
    __shared__ double sm[3][RB];
    const int t = threadIdx.x;
    const int64_t b = offsets[blockIdx.x], e = offsets[blockIdx.x + 1];
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int64_t i = b + t; i < e; i += RB) {
        p0 += m[i] * vx[i];
        p1 += m[i] * vy[i];
        p2 += m[i] * vz[i];
    }
    sm[0][t] = p0;
    sm[1][t] = p1;
    sm[2][t] = p2;
    __syncthreads();
    for (int h = RB / 2; h > 0; h >>= 1) {
        if (t < h) {
            sm[0][t] += sm[0][t + h];
            sm[1][t] += sm[1][t + h];
            sm[2][t] += sm[2][t + h];
        }
        __syncthreads();
    }
    if (t < 3) P[(size_t)blockIdx.x * 3 + t] = sm[t][0];
}

__global__ __launch_bounds__(RB) void k_hc_apply_b(double *x, double *y, double *z, int64_t n,
                                                   const int32_t *sysid, const double *P,
                                                   const double *m_star, const double *dt,
                                                   double hfac)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    const int s = sysid[i];
    const double h = hfac * dt[s];
    x[i] += (h * P[(size_t)s * 3 + 0]) / m_star[s];
    y[i] += (h * P[(size_t)s * 3 + 1]) / m_star[s];
    z[i] += (h * P[(size_t)s * 3 + 2]) / m_star[s];
}

__global__ __launch_bounds__(RB) void k_drift_b(double *x, double *y, double *z, double *vx,
                                                double *vy, double *vz, int64_t n,
                                                const int32_t *sysid, double G,
                                                const double *m_star, const double *dt,
                                                double hfac, int32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    const int s = sysid[i];
    double X = x[i], Y = y[i], Z = z[i], VX = vx[i], VY = vy[i], VZ = vz[i];
    const int st = kepler_uv(G * m_star[s], hfac * dt[s], X, Y, Z, VX, VY, VZ);
    if (st) atomicOr(status, st);
    x[i] = X; y[i] = Y; z[i] = Z;
    vx[i] = VX; vy[i] = VY; vz[i] = VZ;
}

hipError_t launch_rcrit_b(const genga_bodies *b, const BatchDev &bd, char *ws, hipStream_t s)
{
    const unsigned nb = (unsigned)((b->n + RB - 1) / RB);
    hipLaunchKernelGGL(k_rcrit_b, dim3(nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx, b->vy, b->vz,
                       b->m, b->rc, b->n, bd.sysid, bd.m_star, bd.dt, bd.n1, bd.n2, (int32_t *)ws);
    return hipGetLastError();
}

hipError_t launch_hc_b(genga_bodies *b, const BatchDev &bd, double hfac, hipStream_t s)
{
    hipLaunchKernelGGL(k_momentum_sys, dim3((unsigned)bd.S), dim3(RB), 0, s, b->vx, b->vy, b->vz,
                       b->m, bd.offsets, bd.P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((b->n + RB - 1) / RB);
    hipLaunchKernelGGL(k_hc_apply_b, dim3(nb), dim3(RB), 0, s, b->x, b->y, b->z, b->n, bd.sysid,
                       bd.P, bd.m_star, bd.dt, hfac);
    return hipGetLastError();
}

hipError_t launch_drift_b(genga_bodies *b, const BatchDev &bd, double G, double hfac, char *ws,
                          hipStream_t s)
{
    const unsigned nb = (unsigned)((b->n + RB - 1) / RB);
    hipLaunchKernelGGL(k_drift_b, dim3(nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx, b->vy, b->vz,
                       b->n, bd.sysid, G, bd.m_star, bd.dt, hfac, (int32_t *)ws);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_clear_status(char *ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, (int32_t *)ws);
    return hipGetLastError();
}

hipError_t launch_rcrit(const genga_bodies *b, const genga_params *p, char *ws, hipStream_t s)
{
    const unsigned nb = (unsigned)((b->n + RB - 1) / RB);
    hipLaunchKernelGGL(k_rcrit, dim3(nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx, b->vy, b->vz,
                       b->m, b->rc, b->n, p->m_star, p->dt, p->n1, p->n2, (int32_t *)ws);
    return hipGetLastError();
}

hipError_t launch_hc(genga_bodies *b, double m_star, double h, const Layout &L, char *ws,
                     hipStream_t s, int64_t nsum)
{
    double *hc = (double *)(ws + L.hc);
    hipLaunchKernelGGL(k_momentum_partial, dim3((unsigned)L.nb), dim3(RB), 0, s, b->vx, b->vy,
                       b->vz, b->m, nsum, hc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hc_apply, dim3((unsigned)L.nb), dim3(RB), 0, s, b->x, b->y, b->z, b->n,
                       hc, L.nb, h, m_star);
    return hipGetLastError();
}

// HC(h) with the partials hc_in (the fixed order of k_hc_apply), then the
// Kepler drift, then the block partial of m v of the drifted bodies
// [0, nsum) into hc_out: the Sun kick, the drift and the next Sun kick's
// momentum sum in one pass over the bodies.
__global__ __launch_bounds__(RB) void k_hc_drift(double *x, double *y, double *z, double *vx,
                                                 double *vy, double *vz, const double *m, int64_t n,
                                                 int64_t nsum, const double *hc_in, int64_t nb,
                                                 double h, double m_star, double mu, double dt,
                                                 double *hc_out, int32_t *status)
{
    __shared__ double sm[3][RB];
    const int t = threadIdx.x;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int64_t b = t; b < nb; b += RB) {
        p0 += hc_in[b * 3 + 0];
        p1 += hc_in[b * 3 + 1];
        p2 += hc_in[b * 3 + 2];
    }
    sm[0][t] = p0;
    sm[1][t] = p1;
    sm[2][t] = p2;
    __syncthreads();
    for (int hh = RB / 2; hh > 0; hh >>= 1) {
        if (t < hh) {
            sm[0][t] += sm[0][t + hh];
            sm[1][t] += sm[1][t + hh];
            sm[2][t] += sm[2][t + hh];
        }
        __syncthreads();
    }
    const double P0 = sm[0][0], P1 = sm[1][0], P2 = sm[2][0];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * RB + t;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    if (i < n) {
        double X = x[i] + (h * P0) / m_star, Y = y[i] + (h * P1) / m_star,
               Z = z[i] + (h * P2) / m_star;
        double VX = vx[i], VY = vy[i], VZ = vz[i];
        const int st = kepler_uv(mu, dt, X, Y, Z, VX, VY, VZ);
        if (st) atomicOr(status, st);
        x[i] = X; y[i] = Y; z[i] = Z;
        vx[i] = VX; vy[i] = VY; vz[i] = VZ;
        if (i < nsum) {
            const double mi = m[i];
            q0 = mi * VX;
            q1 = mi * VY;
            q2 = mi * VZ;
        }
    }
    sm[0][t] = q0;
    sm[1][t] = q1;
    sm[2][t] = q2;
    __syncthreads();
    for (int hh = RB / 2; hh > 0; hh >>= 1) {
        if (t < hh) {
            sm[0][t] += sm[0][t + hh];
            sm[1][t] += sm[1][t + hh];
            sm[2][t] += sm[2][t + hh];
        }
        __syncthreads();
    }
    if (t < 3) hc_out[(size_t)blockIdx.x * 3 + t] = sm[t][0];
}

hipError_t launch_momentum(const genga_bodies *b, const Layout &L, char *ws, hipStream_t s,
                           int64_t nsum)
{
    hipLaunchKernelGGL(k_momentum_partial, dim3((unsigned)L.nb), dim3(RB), 0, s, b->vx, b->vy,
                       b->vz, b->m, nsum, (double *)(ws + L.hc));
    return hipGetLastError();
}

hipError_t launch_hc_drift(genga_bodies *b, double m_star, double h, double mu, double dt,
                           const Layout &L, char *ws, hipStream_t s, int64_t nsum)
{
    hipLaunchKernelGGL(k_hc_drift, dim3((unsigned)L.nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx,
                       b->vy, b->vz, b->m, b->n, nsum, (const double *)(ws + L.hc), L.nb, h,
                       m_star, mu, dt, (double *)(ws + L.hc2), (int32_t *)ws);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Post-Newtonian term (Sect. 3, eq. apn) by the implicit midpoint rule (eq.
// implicit) in heliocentric velocities u = v + P / m_star.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void apn(double mu, double eta, double c2, const double X[3],
                                    const double U[3], double A[3])
{
    const double r = __builtin_sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
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

// Sum of the per-block partials (stride w, component c) in a fixed tree order.
__device__ __forceinline__ double block_sum_partials(const double *part, int64_t nb, int w, int c,
                                                     double *sm)
{
    const int t = threadIdx.x;
    double v = 0.0;
    for (int64_t b = t; b < nb; b += RB) v += part[b * w + c];
    __syncthreads();
    sm[t] = v;
    __syncthreads();
    for (int hh = RB / 2; hh > 0; hh >>= 1) {
        if (t < hh) sm[t] += sm[t + hh];
        __syncthreads();
    }
    return sm[0];
}

// u' of every body (into gru) and per-block partials of m u' and m.
__global__ __launch_bounds__(RB) void k_gr_update(const double *x, const double *y, const double *z,
                                                  const double *vx, const double *vy,
                                                  const double *vz, const double *m, int64_t n,
                                                  int64_t npad, const double *hc, int64_t nb,
                                                  double G, double m_star, double c2, double h,
                                                  double *gru, double *grp, int32_t *status)
{
    __shared__ double sm[RB];
    __shared__ double red[4][RB];
    double P[3];
    for (int c = 0; c < 3; ++c) P[c] = block_sum_partials(hc, nb, 3, c, sm);
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * RB + t;
    double U1[3] = {0.0, 0.0, 0.0}, mi = 0.0;
    if (i < n) {
        mi = m[i];
        const double mu = G * (m_star + mi);
        const double eta = m_star * mi / ((m_star + mi) * (m_star + mi));
        const double X[3] = {x[i], y[i], z[i]};
        const double U[3] = {vx[i] + P[0] / m_star, vy[i] + P[1] / m_star, vz[i] + P[2] / m_star};
        double A[3], W[3];
        apn(mu, eta, c2, X, U, A);
        for (int k = 0; k < 3; ++k) U1[k] = U[k] + h * A[k];
        for (int it = 0; it < 50; ++it) {
            for (int k = 0; k < 3; ++k) W[k] = 0.5 * (U[k] + U1[k]);
            apn(mu, eta, c2, X, W, A);
            double d = 0.0, s2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double nk = U[k] + h * A[k];
                d += (nk - U1[k]) * (nk - U1[k]);
                s2 += nk * nk;
                U1[k] = nk;
            }
            if (d <= 1e-32 * s2) break;
        }
        if (!(isfinite(U1[0]) && isfinite(U1[1]) && isfinite(U1[2]))) atomicOr(status, ST_NONFINITE);
        for (int k = 0; k < 3; ++k) gru[(size_t)k * npad + i] = U1[k];
    }
    for (int k = 0; k < 3; ++k) red[k][t] = mi * U1[k];
    red[3][t] = mi;
    __syncthreads();
    for (int hh = RB / 2; hh > 0; hh >>= 1) {
        if (t < hh)
            for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + hh];
        __syncthreads();
    }
    if (t < 4) grp[(size_t)blockIdx.x * 4 + t] = red[t][0];
}

// v_i = u'_i - P' / m_star, P' = sum m u' / (1 + M / m_star).
__global__ __launch_bounds__(RB) void k_gr_apply(double *vx, double *vy, double *vz, int64_t n,
                                                 int64_t npad, const double *gru,
                                                 const double *grp, int64_t nb, double m_star)
{
    __shared__ double sm[RB];
    double Q[3];
    for (int c = 0; c < 3; ++c) Q[c] = block_sum_partials(grp, nb, 4, c, sm);
    const double M = block_sum_partials(grp, nb, 4, 3, sm);
    for (int c = 0; c < 3; ++c) Q[c] /= 1.0 + M / m_star;
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    vx[i] = gru[i] - Q[0] / m_star;
    vy[i] = gru[npad + i] - Q[1] / m_star;
    vz[i] = gru[2 * npad + i] - Q[2] / m_star;
}

hipError_t launch_gr(genga_bodies *b, const genga_params *p, double h, const Layout &L, char *ws,
                     hipStream_t s)
{
    double *hc = (double *)(ws + L.hc);
    double *gru = (double *)(ws + L.gru), *grp = (double *)(ws + L.grp);
    hipLaunchKernelGGL(k_momentum_partial, dim3((unsigned)L.nb), dim3(RB), 0, s, b->vx, b->vy,
                       b->vz, b->m, b->n, hc);
    hipLaunchKernelGGL(k_gr_update, dim3((unsigned)L.nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx,
                       b->vy, b->vz, b->m, b->n, L.npad, hc, L.nb, p->G, p->m_star,
                       p->c_light * p->c_light, h, gru, grp, (int32_t *)ws);
    hipLaunchKernelGGL(k_gr_apply, dim3((unsigned)L.nb), dim3(RB), 0, s, b->vx, b->vy, b->vz, b->n,
                       L.npad, gru, grp, L.nb, p->m_star);
    return hipGetLastError();
}

hipError_t launch_drift(genga_bodies *b, double mu, double dt, char *ws, hipStream_t s)
{
    const unsigned nb = (unsigned)((b->n + RB - 1) / RB);
    hipLaunchKernelGGL(k_drift, dim3(nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx, b->vy, b->vz,
                       b->n, mu, dt, (int32_t *)ws);
    return hipGetLastError();
}

}  // namespace genga
