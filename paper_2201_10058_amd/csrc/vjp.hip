// Adjoint (vector-Jacobian products) of the operators of the base step.
//
// Kick (interaction part H_B, GENGA II Sect. 2 eq. Hb; changeover of Sect. 6.2):
//   a_k = G sum_{j != k} m_j w_kj d_kj,  d_kj = x_j - x_k,  w = K(y) / r^3,
//   y = (r - 0.1 rho) / (0.9 rho),  rho = max(rc_k, rc_j).
// With J_kj = w I + (w_r / r) d d^T (symmetric in k, j) and u = m_k abar_j - m_j abar_k:
//   xbar_k  = G sum_j J_kj u            = G sum_j [ w u + (w_r / r)(d.u) d ]
//   mbar_k  = -G sum_j w d.abar_j
//   rcbar_k = G sum_{j: k owns rho_kj} K'(y) / (0.9 rho^2 r^2) d.u
// where w_r / r = K'/(0.9 rho r^4) - 3K / r^5 and "k owns rho" means rc_k > rc_j,
// or rc_k == rc_j and k < j.  Each row gathers over all columns (no scatter,
// no atomics); the K' terms only arise inside the band 0.1 rho < r < rho,
// which the same candidate test as the kick routes to a slow path.
// The row sums are gathered as
//   sum_j w u = m_k sum_j w abar_j - abar_k sum_j w m_j,
//   d.u = m_k d.abar_j - m_j d.abar_k,
// so no per-pair u is formed.
// HC (eq. Hc), critical radii (eq. rcrit) and the Kepler drift adjoints are
// per body (drift: csrc/kepler.h, kepler_uv_vjp).
#include "device_common.h"
#include "genga_internal.h"
#include "kepler.h"

namespace genga {

struct VjpDev {
    const double *x, *y, *z, *m, *rc;
    const double *abx, *aby, *abz;
    double scale;         // abar = scale * (abx, aby, abz)
    int64_t n, npad, slice_len;
    int gx;
    double *part;         // [slices][5][npad]: xbar (3), -mbar / G, rcbar / G
    int32_t *status;
    double c53, c75;      // 5/3 and 7/5
};

template <int NT>
struct VjpSmem {
    double4 xyzm[NT];     // x_j, y_j, z_j, 3/2 m_j
    double4 abr[NT];      // 3/2 scale * abar_j (3), rc_j^2
    double rc[NT];        // rc_j
};

// Fast-path weights to first order in e = 1 - r2 y^2 (y = v_rsq_f64(r2),
// |e| < 1.1e-7; the neglected second-order terms are below 6e-14 relative):
//   r^-3 = y^3 (1 + 3/2 e) = 3/2 y^3 (5/3 - r2 y^2)
//   r^-5 = y^5 (1 + 5/2 e) = 5/2 y^5 (7/5 - r2 y^2).
// Column values are staged times 3/2 (M_j = 3/2 m_j, AB_j = 3/2 abar_j), so
// with w = y^3 (5/3 - r2 y^2) = r^-3 / (3/2) the products w AB_j, w M_j and
// w d.AB_j are the exact terms, du = m_k d.AB_j - M_j d.abar_k = 3/2 d.u, and
// c = y^5 (7/5 - r2 y^2) du = 3/5 r^-5 d.u, whose sum B enters xbar as -5 B
// (the fast-path w_r / r is -3 r^-5).  The slow path stores w and c in the
// same units.
template <int NT>
__global__ __launch_bounds__(NT) void k_kick_vjp(VjpDev a)
{
    __shared__ VjpSmem<NT> sm;
    const int tid = threadIdx.x;
    const int64_t bx = blockIdx.x, s = blockIdx.y;
    const int64_t k = bx * NT + tid;
    const int64_t j0 = s * a.slice_len;
    const int64_t j1 = min(a.n, j0 + a.slice_len);
    const int vzero = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
    const double c53 = a.c53 + (double)vzero, c75 = a.c75 + (double)vzero;
    const double4 *t_xyzm = sm.xyzm + vzero;
    const double4 *t_abr = sm.abr + vzero;
    const double *t_rc = sm.rc + vzero;

    const bool valid = k < a.n;
    double xk, yk, zk, mk = 0.0, rck = 0.0, rc2k = 0.0, abxk = 0.0, abyk = 0.0, abzk = 0.0;
    if (valid) {
        xk = a.x[k]; yk = a.y[k]; zk = a.z[k];
        mk = a.m[k];
        rck = a.rc[k];
        rc2k = rck * rck;
        abxk = a.scale * a.abx[k];
        abyk = a.scale * a.aby[k];
        abzk = a.scale * a.abz[k];
    } else {
        xk = yk = zk = __builtin_nan("");
    }
    // (3/2-scaled) sums: SA = sum w abar_j, SW = sum w m_j, Mb = sum w d.abar_j,
    // B = sum c d; xbar = mk SA - abar_k SW - 5 B (scales undone at the end).
    double SAx = 0, SAy = 0, SAz = 0, SW = 0, Bx = 0, By = 0, Bz = 0, Mb = 0, Rb = 0;

    for (int64_t t0 = j0; t0 < j1; t0 += NT) {
        __syncthreads();
        {
            const int64_t jg = t0 + tid;
            if (jg < j1) {
                const double rcj = a.rc[jg];
                if (!(rcj >= 0.0 && rcj < INFINITY)) atomicOr(a.status, ST_RCRIT);
                const double sc = 1.5 * a.scale;
                sm.xyzm[tid] = make_double4(a.x[jg], a.y[jg], a.z[jg], 1.5 * a.m[jg]);
                sm.abr[tid] = make_double4(sc * a.abx[jg], sc * a.aby[jg], sc * a.abz[jg],
                                           rcj * rcj);
                sm.rc[tid] = rcj;
            }
        }
        __syncthreads();
        const int tn = (int)min((int64_t)NT, j1 - t0);
        for (int jj = 0; jj < tn; ++jj) {
            const double4 b = t_xyzm[jj];
            const double4 ab = t_abr[jj];
            const double dx = b.x - xk, dy = b.y - yk, dz = b.z - zk;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const bool cand = r2 <= vmax_f64(rc2k, ab.w);
            const double yv = __builtin_amdgcn_rsq(r2);
            const double y2 = yv * yv;
            const double p3 = __builtin_fma(-r2, y2, c53);
            const double p5 = __builtin_fma(-r2, y2, c75);
            const double y3 = y2 * yv;
            double w = y3 * p3;                       // r^-3 / (3/2)
            const double da = __builtin_fma(dz, ab.z, __builtin_fma(dy, ab.y, dx * ab.x));
            const double db = __builtin_fma(dz, abzk, __builtin_fma(dy, abyk, dx * abxk));
            const double du = __builtin_fma(mk, da, -(b.w * db));   // 3/2 d.u
            double cq = ((y3 * y2) * p5) * du;                      // 3/5 r^-5 d.u
            if (cand) {
                const int64_t jg = t0 + jj;
                w = 0.0;
                cq = 0.0;
                if (jg != k) {
                    if (r2 == 0.0) {
                        atomicOr(a.status, ST_NONFINITE);
                    } else {
                        // as in the kick's rare path: 1/r from one corrected
                        // v_rsq_f64, 1/rho by v_rcp_f64 and Newton steps, no
                        // IEEE division and no global memory access
                        const double rcj = t_rc[jj];
                        const double y0 = __builtin_amdgcn_rsq(r2);
                        const double e0 = __builtin_fma(-r2, y0 * y0, 1.0);
                        const double yc = __builtin_fma(y0 * e0, 0.5, y0);    // 1 / r
                        const double yc2 = yc * yc, yc3 = yc2 * yc;
                        double K = 1.0, Kp = 0.0, irho = 0.0;
                        if (r2 < rho2_of(rck, rcj)) {
                            const double rho = rck > rcj ? rck : rcj;
                            irho = __builtin_amdgcn_rcp(rho);
                            irho = __builtin_fma(irho, __builtin_fma(-rho, irho, 1.0), irho);
                            irho = __builtin_fma(irho, __builtin_fma(-rho, irho, 1.0), irho);
                            changeover_kdk_of_y(
                                __builtin_fma((r2 * yc) * irho, 1.0 / 0.9, -1.0 / 9.0), K, Kp);
                        }
                        // fast-path units: w = (K / r^3) / (3/2) and
                        // -5 c = (w_r / r) d.u with du = 3/2 d.u, where
                        // w_r / r = K' / (0.9 rho r^4) - 3 K / r^5
                        w = (K * yc3) * (2.0 / 3.0);
                        const double wr_r =
                            (Kp * (irho * (1.0 / 0.9))) * (yc2 * yc2) - (3.0 * K) * (yc3 * yc2);
                        cq = -(wr_r * du) * (1.0 / 7.5);
                        const bool owner = rck > rcj || (rck == rcj && k < jg);
                        if (owner && Kp != 0.0)
                            Rb += ((Kp * (irho * irho)) * (1.0 / 0.9)) * yc2 * (du * (2.0 / 3.0));
                    }
                }
            }
            SAx = __builtin_fma(w, ab.x, SAx);
            SAy = __builtin_fma(w, ab.y, SAy);
            SAz = __builtin_fma(w, ab.z, SAz);
            SW = __builtin_fma(w, b.w, SW);
            Mb = __builtin_fma(w, da, Mb);
            Bx = __builtin_fma(cq, dx, Bx);
            By = __builtin_fma(cq, dy, By);
            Bz = __builtin_fma(cq, dz, Bz);
        }
    }
    if (valid) {
        // xbar = m_k sum w abar_j - abar_k sum w m_j + sum (w_r / r) d.u d
        double *P = a.part + (size_t)s * 5 * a.npad;
        P[0 * a.npad + k] = __builtin_fma(-5.0, Bx, __builtin_fma(mk, SAx, -(abxk * SW)));
        P[1 * a.npad + k] = __builtin_fma(-5.0, By, __builtin_fma(mk, SAy, -(abyk * SW)));
        P[2 * a.npad + k] = __builtin_fma(-5.0, Bz, __builtin_fma(mk, SAz, -(abzk * SW)));
        P[3 * a.npad + k] = Mb;
        P[4 * a.npad + k] = Rb;
    }
}

__global__ __launch_bounds__(RB) void k_kick_vjp_reduce(const double *part, int64_t n, int64_t npad,
                                                        int slices, double G, double *xb,
                                                        double *yb, double *zb, double *mb,
                                                        double *rcb)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    double acc[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        acc[c] = ordered_sum(part + (size_t)c * npad + i, (size_t)5 * npad, slices);
    }
    xb[i] += G * acc[0];
    yb[i] += G * acc[1];
    zb[i] += G * acc[2];
    mb[i] -= G * acc[3];
    rcb[i] += G * acc[4];
}

// rc = max(n1 R_H, n2 |dt| |v|), R_H = |x| (m / 3 m_star)^(1/3); ties -> Hill term.
__global__ __launch_bounds__(RB) void k_rcrit_vjp(const double *x, const double *y, const double *z,
                                                  const double *vx, const double *vy,
                                                  const double *vz, const double *m, int64_t n,
                                                  double m_star, double dt, double n1, double n2,
                                                  genga_adjoint adj)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    const double rb = adj.rc[i];
    if (rb == 0.0) return;
    const double r = __builtin_sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
    const double v = __builtin_sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    const double q = cbrt(m[i] / (3.0 * m_star));
    const double a = n1 * r * q;
    const double b = n2 * fabs(dt) * v;
    if (a >= b) {
        if (r > 0.0) {
            const double f = rb * n1 * q / r;
            adj.x[i] += f * x[i];
            adj.y[i] += f * y[i];
            adj.z[i] += f * z[i];
        }
        if (m[i] > 0.0) adj.m[i] += rb * a / (3.0 * m[i]);
    } else if (v > 0.0) {
        const double f = rb * n2 * fabs(dt) / v;
        adj.vx[i] += f * vx[i];
        adj.vy[i] += f * vy[i];
        adj.vz[i] += f * vz[i];
    }
}

// HC: x_out = x_in + h P / m_star, P = sum m v.  With S = sum_i xbar_i:
//   vbar_j += (h m_j / m_star) S,  mbar_j += (h / m_star) v_j . S.
__global__ __launch_bounds__(RB) void k_sum3_partial(const double *a, const double *b,
                                                     const double *c, int64_t n, double *out)
{
    __shared__ double sm[3][RB];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * RB + t;
    sm[0][t] = i < n ? a[i] : 0.0;
    sm[1][t] = i < n ? b[i] : 0.0;
    sm[2][t] = i < n ? c[i] : 0.0;
    __syncthreads();
    for (int h = RB / 2; h > 0; h >>= 1) {
        if (t < h) {
            sm[0][t] += sm[0][t + h];
            sm[1][t] += sm[1][t + h];
            sm[2][t] += sm[2][t + h];
        }
        __syncthreads();
    }
    if (t < 3) out[(size_t)blockIdx.x * 3 + t] = sm[t][0];
}

__global__ __launch_bounds__(RB) void k_hc_vjp_apply(const double *vx, const double *vy,
                                                     const double *vz, const double *m, int64_t n,
                                                     const double *part, int64_t nb, double h,
                                                     double m_star, genga_adjoint adj)
{
    __shared__ double sm[3][RB];
    const int t = threadIdx.x;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int64_t b = t; b < nb; b += RB) {
        p0 += part[b * 3 + 0];
        p1 += part[b * 3 + 1];
        p2 += part[b * 3 + 2];
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
    const double S0 = sm[0][0], S1 = sm[1][0], S2 = sm[2][0];
    const double f = h * m[i] / m_star;
    adj.vx[i] += f * S0;
    adj.vy[i] += f * S1;
    adj.vz[i] += f * S2;
    adj.m[i] += (h / m_star) * (vx[i] * S0 + vy[i] * S1 + vz[i] * S2);
}

__global__ __launch_bounds__(RB) void k_drift_vjp(const double *x, const double *y, const double *z,
                                                  const double *vx, const double *vy,
                                                  const double *vz, int64_t n, double mu,
                                                  double dt, genga_adjoint adj, int32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= n) return;
    const double X[3] = {x[i], y[i], z[i]}, V[3] = {vx[i], vy[i], vz[i]};
    double xb[3] = {adj.x[i], adj.y[i], adj.z[i]}, vb[3] = {adj.vx[i], adj.vy[i], adj.vz[i]};
    const int st = kepler_uv_vjp(mu, dt, X, V, xb, vb);
    if (st) atomicOr(status, st);
    adj.x[i] = xb[0]; adj.y[i] = xb[1]; adj.z[i] = xb[2];
    adj.vx[i] = vb[0]; adj.vy[i] = vb[1]; adj.vz[i] = vb[2];
}

// ---------------------------------------------------------------------------
hipError_t launch_kick_vjp(const genga_bodies *b, const genga_params *p, double scale,
                           const double *abx, const double *aby, const double *abz,
                           genga_adjoint *adj, char *ws, hipStream_t s)
{
    KickCfg c = choose_kick_cfg(b->n, p);
    if (c.use_sym) {
        // the symmetric form, where the kick takes it (csrc/vjp_sym.hip)
        const Layout L = make_layout(b->n, c);
        return launch_kick_vjp_sym(c.sym, b, p->G, scale, abx, aby, abz, adj,
                                   (double *)(ws + L.part), (int32_t *)(ws + L.status), s);
    }
    // one row per thread for the adjoint (its register footprint is larger)
    c.ipt = 1;
    c.gx = (int)((b->n + KB - 1) / KB);
    const Layout L = make_layout(b->n, c);
    VjpDev d;
    d.x = b->x; d.y = b->y; d.z = b->z; d.m = b->m; d.rc = b->rc;
    d.abx = abx; d.aby = aby; d.abz = abz;
    d.scale = scale;
    d.n = b->n;
    d.npad = L.npad;
    d.slice_len = c.slice_len;
    d.gx = c.gx;
    d.part = (double *)(ws + L.part);
    d.status = (int32_t *)(ws + L.status);
    d.c53 = 5.0 / 3.0;
    d.c75 = 7.0 / 5.0;
    hipLaunchKernelGGL(k_kick_vjp<KB>, dim3(c.gx, c.slices), dim3(KB), 0, s, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kick_vjp_reduce, dim3((unsigned)L.nb), dim3(RB), 0, s, d.part, b->n,
                       L.npad, c.slices, p->G, adj->x, adj->y, adj->z, adj->m, adj->rc);
    return hipGetLastError();
}

hipError_t launch_rcrit_vjp(const genga_bodies *b, const genga_params *p, genga_adjoint *adj,
                            hipStream_t s)
{
    const unsigned nb = (unsigned)((b->n + RB - 1) / RB);
    hipLaunchKernelGGL(k_rcrit_vjp, dim3(nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx, b->vy,
                       b->vz, b->m, b->n, p->m_star, p->dt, p->n1, p->n2, *adj);
    return hipGetLastError();
}

hipError_t launch_hc_vjp(const genga_bodies *b, const genga_params *p, double h, genga_adjoint *adj,
                         const Layout &L, char *ws, hipStream_t s)
{
    double *part = (double *)(ws + L.hc);
    hipLaunchKernelGGL(k_sum3_partial, dim3((unsigned)L.nb), dim3(RB), 0, s, adj->x, adj->y,
                       adj->z, b->n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hc_vjp_apply, dim3((unsigned)L.nb), dim3(RB), 0, s, b->vx, b->vy, b->vz,
                       b->m, b->n, part, L.nb, h, p->m_star, *adj);
    return hipGetLastError();
}

hipError_t launch_drift_vjp(const genga_bodies *b, const genga_params *p, double dt,
                            genga_adjoint *adj, char *ws, hipStream_t s)
{
    const unsigned nb = (unsigned)((b->n + RB - 1) / RB);
    hipLaunchKernelGGL(k_drift_vjp, dim3(nb), dim3(RB), 0, s, b->x, b->y, b->z, b->vx, b->vy,
                       b->vz, b->n, p->G * p->m_star, dt, *adj, (int32_t *)ws);
    return hipGetLastError();
}

}  // namespace genga
