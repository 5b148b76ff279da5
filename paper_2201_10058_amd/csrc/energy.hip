// Total energy of the democratic heliocentric splitting (GENGA II Sect. 2,
// eqs. H, Ha, Hb, Hc), in binary64:
//   T   = sum_i m_i |v_i|^2 / 2                      (kinetic part of H_A)
//   U_* = -G m_star sum_i m_i / |x_i|                (Kepler part of H_A)
//   U   = -G sum_{i<j} m_i m_j / r_ij                (H_B without changeover)
//   C   = |sum_i m_i v_i|^2 / (2 m_star)             (H_C)
// U is evaluated as -G/2 sum_i m_i phi_i, phi_i = sum_{j != i} m_j / r_ij,
// with the rows x column-slices tiling of the kick (columns staged in LDS).
// Every sum after the pair loop runs in a fixed order, so the result does not
// depend on scheduling.
#include <math.h>

#include "device_common.h"
#include "genga_internal.h"

namespace genga {

namespace {

constexpr int EB = 256;   // rows per block of the pair-potential kernel

struct EnergyDev {
    const double *x, *y, *z, *m;
    int64_t n, npad, slice_len;
    double *phi;          // [slices][npad]
    int32_t *status;
};

// phi partial of row i over the columns of slice blockIdx.y.
__global__ __launch_bounds__(EB) void k_energy_phi(EnergyDev a)
{
    __shared__ double4 sm[EB];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * EB + tid;
    const int64_t j0 = (int64_t)blockIdx.y * a.slice_len;
    const int64_t j1 = min(a.n, j0 + a.slice_len);
    double xi, yi, zi;
    if (i < a.n) {
        xi = a.x[i]; yi = a.y[i]; zi = a.z[i];
    } else {
        xi = yi = zi = __builtin_nan("");   // r2 is NaN: no term, no status
    }
    double phi = 0.0;
    bool coincident = false;
    for (int64_t t0 = j0; t0 < j1; t0 += EB) {
        __syncthreads();
        const int64_t jg = t0 + tid;
        if (jg < j1) sm[tid] = make_double4(a.x[jg], a.y[jg], a.z[jg], a.m[jg]);
        __syncthreads();
        const int tn = (int)min((int64_t)EB, j1 - t0);
        for (int jj = 0; jj < tn; ++jj) {
            const double4 b = sm[jj];
            const double dx = b.x - xi, dy = b.y - yi, dz = b.z - zi;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            // 1/r from v_rsq_f64 with one Newton correction: y (1 + e/2),
            // e = 1 - r2 y^2; the remainder 3/8 e^2 is below 5e-15.
            const double y = __builtin_amdgcn_rsq(r2);
            const double e = __builtin_fma(-r2, y * y, 1.0);
            const double rinv = __builtin_fma(y * e, 0.5, y);
            if (r2 > 0.0) {
                phi = __builtin_fma(b.w, rinv, phi);
            } else if (r2 == 0.0 && t0 + jj != i) {
                coincident = true;
            }
        }
    }
    if (coincident) atomicOr(a.status, ST_NONFINITE);
    if (i < a.n) a.phi[(size_t)blockIdx.y * a.npad + i] = phi;
}

// Per-block sums of the six per-body terms (T, U_*, U, P) in a fixed tree.
__global__ __launch_bounds__(RB) void k_energy_rows(const double *x, const double *y,
                                                    const double *z, const double *vx,
                                                    const double *vy, const double *vz,
                                                    const double *m, const double *phi,
                                                    int64_t n, int64_t npad, int slices, double G,
                                                    double m_star, double *bpart)
{
    __shared__ double sm[6][RB];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * RB + t;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const double p = ordered_sum(phi + i, (size_t)npad, slices);
        const double mi = m[i];
        const double v2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
        const double r = __builtin_sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
        v[0] = 0.5 * mi * v2;
        v[1] = -G * m_star * mi / r;
        v[2] = -0.5 * G * mi * p;
        v[3] = mi * vx[i];
        v[4] = mi * vy[i];
        v[5] = mi * vz[i];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) sm[c][t] = v[c];
    __syncthreads();
    for (int h = RB / 2; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int c = 0; c < 6; ++c) sm[c][t] += sm[c][t + h];
        }
        __syncthreads();
    }
    if (t < 6) bpart[(size_t)blockIdx.x * 6 + t] = sm[t][0];
}

// One block: the block sums in a fixed order, then out = (E, T, U_*, U, C).
__global__ __launch_bounds__(RB) void k_energy_final(const double *bpart, int64_t nb,
                                                     double m_star, double *out)
{
    __shared__ double sm[6][RB];
    const int t = threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = t; b < nb; b += RB) {
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] += bpart[b * 6 + c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) sm[c][t] = v[c];
    __syncthreads();
    for (int h = RB / 2; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int c = 0; c < 6; ++c) sm[c][t] += sm[c][t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double T = sm[0][0], Us = sm[1][0], U = sm[2][0];
        const double P2 = sm[3][0] * sm[3][0] + sm[4][0] * sm[4][0] + sm[5][0] * sm[5][0];
        const double C = P2 / (2.0 * m_star);
        out[0] = T + Us + U + C;
        out[1] = T;
        out[2] = Us;
        out[3] = U;
        out[4] = C;
    }
}

// Gauss-Legendre rule of 32 points on [-1, 1].
struct GL32 {
    double x[32], w[32];
};

constexpr int EP = 256;     // threads per block of the pair correction
constexpr int EPG = 512;    // blocks of the pair correction (fixed grid)

// E_K - E over the listed pairs inside rho_ij:
//   G m_i m_j (1/r - 1/rho - int_{max(r, 0.1 rho)}^{rho} K(s)/s^2 ds),
// the integral by the 32-point Gauss-Legendre rule (K is smooth between the
// band edges, the only points where its second derivative jumps).  Block
// partials in a fixed order (fixed grid).
__global__ __launch_bounds__(EP) void k_energy_pairs(const int32_t *pi, const int32_t *pj,
                                                     const int64_t *cnt, int64_t cap,
                                                     const double *x, const double *y,
                                                     const double *z, const double *m,
                                                     const double *rc, double G, GL32 gl,
                                                     double *part)
{
    __shared__ double sm[EP];
    const int t = threadIdx.x;
    const int64_t c = *cnt;
    const int64_t np = c < cap ? c : cap;
    double acc = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * EP + t; q < np; q += (int64_t)gridDim.x * EP) {
        const int64_t i = pi[q], j = pj[q];
        const double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const double rho = rc[i] > rc[j] ? rc[i] : rc[j];
        if (!(r2 < rho * rho) || r2 == 0.0) continue;
        const double r = __builtin_sqrt(r2);
        const double a = r > 0.1 * rho ? r : 0.1 * rho;
        const double half = 0.5 * (rho - a), mid = 0.5 * (rho + a);
        double I = 0.0;
        for (int k = 0; k < 32; ++k) {
            const double sk = mid + half * gl.x[k];
            I += gl.w[k] * changeover_k(sk, rho) / (sk * sk);
        }
        I *= half;
        acc += G * m[i] * m[j] * (1.0 / r - 1.0 / rho - I);
    }
    sm[t] = acc;
    __syncthreads();
    for (int h = EP / 2; h > 0; h >>= 1) {
        if (t < h) sm[t] += sm[t + h];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(EP) void k_energy_k_final(const double *part, double *out)
{
    __shared__ double sm[EP];
    const int t = threadIdx.x;
    double v = 0.0;
    for (int b = t; b < EPG; b += EP) v += part[b];
    sm[t] = v;
    __syncthreads();
    for (int h = EP / 2; h > 0; h >>= 1) {
        if (t < h) sm[t] += sm[t + h];
        __syncthreads();
    }
    if (t == 0) out[5] = out[0] + sm[0];
}

// Nodes by Newton's method on the Legendre polynomial P_32 from the usual
// cosine guesses; weights 2 / ((1 - x^2) P_32'(x)^2).
GL32 make_gl32()
{
    GL32 g;
    const int n = 32;
    for (int k = 0; k < n / 2; ++k) {
        double xk = cos(M_PI * (k + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = xk;
            for (int l = 2; l <= n; ++l) {
                const double p2 = ((2.0 * l - 1.0) * xk * p1 - (l - 1.0) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (xk * p1 - p0) / (xk * xk - 1.0);
            const double dx = p1 / dp;
            xk -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        const double w = 2.0 / ((1.0 - xk * xk) * dp * dp);
        g.x[k] = -xk;
        g.w[k] = w;
        g.x[n - 1 - k] = xk;
        g.w[n - 1 - k] = w;
    }
    return g;
}

}  // namespace

hipError_t launch_energy_k_pairs(const genga_bodies *b, const genga_params *p, genga_pairs *pairs,
                                 double *out, const Layout &L, char *ws, hipStream_t s)
{
    static const GL32 gl = make_gl32();
    double *part = (double *)(ws + L.part);
    hipLaunchKernelGGL(k_energy_pairs, dim3(EPG), dim3(EP), 0, s, pairs->i, pairs->j, pairs->count,
                       pairs->capacity, b->x, b->y, b->z, b->m, b->rc, p->G, gl, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_k_final, dim3(1), dim3(EP), 0, s, part, out);
    return hipGetLastError();
}

hipError_t launch_energy(const genga_bodies *b, const genga_params *p, double *out,
                         const KickCfg &c, const Layout &L, char *ws, hipStream_t s)
{
    EnergyDev a;
    a.x = b->x; a.y = b->y; a.z = b->z; a.m = b->m;
    a.n = b->n;
    a.npad = L.npad;
    a.slice_len = c.slice_len;
    a.phi = (double *)(ws + L.part);
    a.status = (int32_t *)(ws + L.status);
    const int slices = (int)((b->n + c.slice_len - 1) / c.slice_len);
    // phi takes slices * npad doubles of the partial-sum region (sized for
    // 5 * c.slices * npad); the block sums follow it.
    double *bpart = a.phi + (size_t)slices * L.npad;
    const unsigned gx = (unsigned)((b->n + EB - 1) / EB);
    hipLaunchKernelGGL(k_energy_phi, dim3(gx, (unsigned)slices), dim3(EB), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_rows, dim3((unsigned)L.nb), dim3(RB), 0, s, b->x, b->y, b->z,
                       b->vx, b->vy, b->vz, b->m, a.phi, b->n, L.npad, slices, p->G, p->m_star,
                       bpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(RB), 0, s, bpart, L.nb, p->m_star, out);
    return hipGetLastError();
}

}  // namespace genga
