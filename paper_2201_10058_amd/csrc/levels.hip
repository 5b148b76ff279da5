// Symplectic levels of the base step (GENGA II Sect. 6.2, higher-level
// changeover functions; Appendix A, the recursive encounter routine).
//
// The bodies of an encounter list are advanced, instead of their Kepler
// drift, by sub-steps of a shorter time step: new critical radii (eq. rcrit
// with the sub-step), a kick over the list's pairs with the level weight
//   W_l(r) = prod_{k<l} (1 - K(r; rho_k)) * K(r; rho_l),
// the drift of the list's bodies, and the same kick again; the pairs that are
// closer than the level's critical radius form the next level's list, whose
// bodies are advanced one level deeper instead of that drift.
//
// Everything is sparse over the lists and runs on the device with fixed grids
// that read the list sizes from device memory, so a step has a fixed launch
// sequence (no host synchronisation; capturable).  Lists stay in the
// canonical order (i ascending, then j): the next level's list is a
// stream compaction of the upper one (block counts, one scan, ordered
// writes).  For the kicks every list gets an adjacency structure whose
// partners are sorted ascending per body, so each body adds its pair terms in
// a fixed order and no floating-point atomics are used.
#include "device_common.h"
#include "genga_internal.h"
#include "kepler.h"

namespace genga {

namespace {

constexpr int LT = 256;     // threads per block of the list kernels
constexpr int LG = 1024;    // blocks of the grid-stride list kernels
constexpr int DB = 256;     // blocks (and chunks) of the list compaction
constexpr int ST = 1024;    // threads of the one-block scan of the adjacency tile sums

__device__ __forceinline__ int64_t list_len(const int64_t *cnt, int64_t cap)
{
    const int64_t c = *cnt;
    return c < cap ? c : cap;
}

__device__ __forceinline__ double rho_of(const double *rc, int64_t i, int64_t j)
{
    return rc[i] > rc[j] ? rc[i] : rc[j];
}

// Squared separation with the encounter predicate's operation order.
__device__ __forceinline__ double sep2(const double *x, const double *y, const double *z,
                                       int64_t i, int64_t j)
{
    const double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

__global__ __launch_bounds__(64) void k_level_begin(int64_t *lcount, int L, const int64_t *cnt0)
{
    const int t = threadIdx.x;
    if (t < L) lcount[t] = t == 0 ? *cnt0 : 0;
}

// E_0 to the caller's list: min(count, capacities) entries and the true count.
__global__ __launch_bounds__(LT) void k_copy_pairs(const int32_t *si, const int32_t *sj,
                                                   const int64_t *scnt, int64_t scap, int32_t *di,
                                                   int32_t *dj, int64_t dcap, int64_t *dcnt,
                                                   int32_t *status)
{
    const int64_t c = *scnt;
    int64_t m = c < scap ? c : scap;
    if (m > dcap) m = dcap;
    const int64_t t0 = (int64_t)blockIdx.x * LT + threadIdx.x;
    for (int64_t p = t0; p < m; p += (int64_t)gridDim.x * LT) {
        di[p] = si[p];
        dj[p] = sj[p];
    }
    if (t0 == 0) {
        *dcnt = c;
        if (c > dcap) atomicOr(status, ST_OVERFLOW);
    }
}

__global__ __launch_bounds__(LT) void k_zero_i32(int32_t *a, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * LT + threadIdx.x; k < n; k += (int64_t)gridDim.x * LT)
        a[k] = 0;
}

// ---------------------------------------------------------------------------
// Adjacency of a list: degrees, their scan (offsets and the ascending list of
// bodies), fill in arrival order, and placement of each entry at its rank
// among the body's partners (so every segment is sorted ascending).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LT) void k_adj_count(const int32_t *pi, const int32_t *pj,
                                                  const int64_t *cnt, int64_t cap, int32_t *deg)
{
    const int64_t m = list_len(cnt, cap);
    for (int64_t p = (int64_t)blockIdx.x * LT + threadIdx.x; p < m; p += (int64_t)gridDim.x * LT) {
        atomicAdd(deg + pi[p], 1);
        atomicAdd(deg + pj[p], 1);
    }
}

// Offsets and body list in three passes over tiles of LT bodies: tile sums
// of the degrees and of the bodies with a pair, one block scanning the tile
// sums, and the tiles again with those offsets.
__global__ __launch_bounds__(LT) void k_adj_tiles(const int32_t *deg, int64_t n, int64_t *tsum)
{
    __shared__ int64_t sm[LT / 64];
    const int64_t k = (int64_t)blockIdx.x * LT + threadIdx.x;
    const int32_t d = k < n ? deg[k] : 0;
    int64_t td, tb;
    block_excl_scan<LT>(d, &td, sm);
    block_excl_scan<LT>(d > 0 ? 1 : 0, &tb, sm);
    if (threadIdx.x == 0) {
        tsum[2 * blockIdx.x] = td;
        tsum[2 * blockIdx.x + 1] = tb;
    }
}

__global__ __launch_bounds__(ST) void k_adj_top(int64_t *tsum, int64_t ntiles, int32_t *start,
                                                int64_t n, int32_t *nbod)
{
    __shared__ int64_t sm[ST / 64];
    const int t = threadIdx.x;
    const int64_t ch = (ntiles + ST - 1) / ST;
    const int64_t k0 = min(ntiles, t * ch), k1 = min(ntiles, k0 + ch);
    int64_t sd = 0, sb = 0;
    for (int64_t k = k0; k < k1; ++k) {
        sd += tsum[2 * k];
        sb += tsum[2 * k + 1];
    }
    int64_t td, tb;
    int64_t od = block_excl_scan<ST>(sd, &td, sm);
    int64_t ob = block_excl_scan<ST>(sb, &tb, sm);
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t a = tsum[2 * k], b = tsum[2 * k + 1];
        tsum[2 * k] = od;
        tsum[2 * k + 1] = ob;
        od += a;
        ob += b;
    }
    if (t == 0) {
        start[n] = (int32_t)td;
        *nbod = (int32_t)tb;
    }
}

__global__ __launch_bounds__(LT) void k_adj_write(int32_t *deg, int64_t n, const int64_t *tsum,
                                                  int32_t *start, int32_t *bodies)
{
    __shared__ int64_t sm[LT / 64];
    const int64_t k = (int64_t)blockIdx.x * LT + threadIdx.x;
    const int32_t d = k < n ? deg[k] : 0;
    int64_t td, tb;
    const int64_t od = block_excl_scan<LT>(d, &td, sm);
    const int64_t ob = block_excl_scan<LT>(d > 0 ? 1 : 0, &tb, sm);
    if (k < n) {
        start[k] = (int32_t)(tsum[2 * blockIdx.x] + od);
        if (d > 0) bodies[tsum[2 * blockIdx.x + 1] + ob] = (int32_t)k;
        deg[k] = 0;   // fill counter of k_adj_fill
    }
}

// Each pair into both bodies' segments, in arrival order (owner recorded).
__global__ __launch_bounds__(LT) void k_adj_fill(const int32_t *pi, const int32_t *pj,
                                                 const int64_t *cnt, int64_t cap,
                                                 const int32_t *start, int32_t *fill, int32_t *tmp,
                                                 int32_t *owner)
{
    const int64_t m = list_len(cnt, cap);
    for (int64_t p = (int64_t)blockIdx.x * LT + threadIdx.x; p < m; p += (int64_t)gridDim.x * LT) {
        const int32_t i = pi[p], j = pj[p];
        const int32_t si = start[i] + atomicAdd(fill + i, 1);
        tmp[si] = j;
        owner[si] = i;
        const int32_t sj = start[j] + atomicAdd(fill + j, 1);
        tmp[sj] = i;
        owner[sj] = j;
    }
}

// Sorted placement: an entry's rank among its body's partners (all distinct)
// is the number of smaller partners in the segment.
__global__ __launch_bounds__(LT) void k_adj_rank(const int32_t *start, int64_t n, const int32_t *tmp,
                                                 const int32_t *owner, int32_t *adj)
{
    const int64_t total = start[n];
    for (int64_t e = (int64_t)blockIdx.x * LT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * LT) {
        const int32_t b = owner[e], v = tmp[e];
        const int32_t s0 = start[b], s1 = start[b + 1];
        int32_t r = 0;
        for (int32_t q = s0; q < s1; ++q) r += tmp[q] < v;
        adj[s0 + r] = v;
    }
}

// ---------------------------------------------------------------------------
// Next level's list: the pairs of list `in` closer than this level's
// critical radius, in the same order.  DB chunks of the input: counts, one
// scan, ordered writes.
// ---------------------------------------------------------------------------
struct DetectDev {
    const int32_t *in_i, *in_j;
    const int64_t *in_cnt;
    int32_t *out_i, *out_j;
    int64_t *out_cnt;
    int64_t *lcount;          // summed sizes of this level's lists
    int64_t cap;
    const double *x, *y, *z, *rc;
    int64_t *bcnt;            // [DB]
};

__device__ __forceinline__ bool detect_pair(const DetectDev &d, int64_t p)
{
    const int64_t i = d.in_i[p], j = d.in_j[p];
    const double rho = rho_of(d.rc, i, j);
    return sep2(d.x, d.y, d.z, i, j) < rho * rho;
}

__device__ __forceinline__ void chunk_of(const DetectDev &d, int64_t &p0, int64_t &p1)
{
    const int64_t m = list_len(d.in_cnt, d.cap);
    const int64_t len = (m + DB - 1) / DB;
    p0 = min(m, (int64_t)blockIdx.x * len);
    p1 = min(m, p0 + len);
}

__global__ __launch_bounds__(LT) void k_detect_count(DetectDev d)
{
    __shared__ int64_t sm[LT / 64];
    int64_t p0, p1;
    chunk_of(d, p0, p1);
    int64_t c = 0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += LT) c += detect_pair(d, p);
    int64_t tot;
    block_excl_scan<LT>(c, &tot, sm);
    if (threadIdx.x == 0) d.bcnt[blockIdx.x] = tot;
}

__global__ __launch_bounds__(DB) void k_detect_scan(DetectDev d)
{
    __shared__ int64_t sm[DB / 64];
    const int64_t v = d.bcnt[threadIdx.x];
    int64_t tot;
    const int64_t ex = block_excl_scan<DB>(v, &tot, sm);
    d.bcnt[threadIdx.x] = ex;
    if (threadIdx.x == 0) {
        *d.out_cnt = tot;
        *d.lcount += tot;
    }
}

__global__ __launch_bounds__(LT) void k_detect_write(DetectDev d)
{
    __shared__ int64_t sm[LT / 64];
    int64_t p0, p1;
    chunk_of(d, p0, p1);
    int64_t run = d.bcnt[blockIdx.x];
    for (int64_t t0 = p0; t0 < p1; t0 += LT) {
        const int64_t p = t0 + threadIdx.x;
        const bool f = p < p1 && detect_pair(d, p);
        int64_t tot;
        const int64_t ex = block_excl_scan<LT>(f ? 1 : 0, &tot, sm);
        if (f) {
            d.out_i[run + ex] = d.in_i[p];
            d.out_j[run + ex] = d.in_j[p];
        }
        run += tot;
    }
}

// ---------------------------------------------------------------------------
// Per-body operators over a list's bodies.
// ---------------------------------------------------------------------------
struct BodyDev {
    const int32_t *bodies;
    const int32_t *nbod;
    double *x, *y, *z, *vx, *vy, *vz;
    const double *m;
    int32_t *status;
};

__global__ __launch_bounds__(LT) void k_rcrit_list(BodyDev a, double *rc, double m_star, double dt,
                                                   double n1, double n2)
{
    const int64_t nb = *a.nbod;
    for (int64_t q = (int64_t)blockIdx.x * LT + threadIdx.x; q < nb; q += (int64_t)gridDim.x * LT) {
        const int32_t i = a.bodies[q];
        const double r = __builtin_sqrt(a.x[i] * a.x[i] + a.y[i] * a.y[i] + a.z[i] * a.z[i]);
        const double v =
            __builtin_sqrt(a.vx[i] * a.vx[i] + a.vy[i] * a.vy[i] + a.vz[i] * a.vz[i]);
        const double rh = r * cbrt(a.m[i] / (3.0 * m_star));
        const double h1 = n1 * rh, h2 = n2 * fabs(dt) * v;
        const double out = h1 > h2 ? h1 : h2;
        if (!(out >= 0.0 && out < INFINITY)) atomicOr(a.status, ST_RCRIT);
        rc[i] = out;
    }
}

__global__ __launch_bounds__(LT) void k_drift_list(BodyDev a, double mu, double dt)
{
    const int64_t nb = *a.nbod;
    for (int64_t q = (int64_t)blockIdx.x * LT + threadIdx.x; q < nb; q += (int64_t)gridDim.x * LT) {
        const int32_t i = a.bodies[q];
        double X = a.x[i], Y = a.y[i], Z = a.z[i], VX = a.vx[i], VY = a.vy[i], VZ = a.vz[i];
        const int st = kepler_uv(mu, dt, X, Y, Z, VX, VY, VZ);
        if (st) atomicOr(a.status, st);
        a.x[i] = X; a.y[i] = Y; a.z[i] = Z;
        a.vx[i] = VX; a.vy[i] = VY; a.vz[i] = VZ;
    }
}

// save = 1: shadow <- state; save = 0: state <- shadow (bodies of the list).
__global__ __launch_bounds__(LT) void k_state_list(BodyDev a, double *shadow, int64_t n, int save)
{
    const int64_t nb = *a.nbod;
    double *c[6] = {a.x, a.y, a.z, a.vx, a.vy, a.vz};
    for (int64_t q = (int64_t)blockIdx.x * LT + threadIdx.x; q < nb; q += (int64_t)gridDim.x * LT) {
        const int32_t i = a.bodies[q];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (save) shadow[(size_t)k * n + i] = c[k][i];
            else c[k][i] = shadow[(size_t)k * n + i];
        }
    }
}

// Kick of level l over a list: v_b += h G sum_j m_j W_l(r_bj) (x_j - x_b) / r^3
// for every body b of the list.  A group of GL lanes takes one body: lane u
// adds the partners u, u + GL, ... of the body's ascending partner list, and
// the GL partial sums are combined by a fixed butterfly, so the result does
// not depend on scheduling.
constexpr int GL = 8;

struct LevelKickDev {
    BodyDev a;
    const int32_t *start, *adj;
    const double *rc[GENGA_MAX_LEVELS];   // rc[0]: level 0 (the bodies' rc)
    int level;
    double G, h;
};

__global__ __launch_bounds__(LT) void k_level_kick(LevelKickDev k)
{
    const BodyDev &a = k.a;
    const int64_t nb = *a.nbod;
    const int u = threadIdx.x & (GL - 1);
    const int64_t g0 = ((int64_t)blockIdx.x * LT + threadIdx.x) / GL;
    const int64_t gstride = (int64_t)gridDim.x * (LT / GL);
    // every lane of a group runs the same trip count (the body loop is
    // uniform per group), so the butterfly below sees all GL lanes
    for (int64_t q = g0; q < nb; q += gstride) {
        const int32_t b = a.bodies[q];
        const double xb = a.x[b], yb = a.y[b], zb = a.z[b];
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int32_t e = k.start[b] + u; e < k.start[b + 1]; e += GL) {
            const int32_t j = k.adj[e];
            const double dx = a.x[j] - xb, dy = a.y[j] - yb, dz = a.z[j] - zb;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            if (r2 == 0.0) {
                atomicOr(a.status, ST_NONFINITE);
                continue;
            }
            const double r = __builtin_sqrt(r2);
            double w = 1.0;
            for (int l = 0; l < k.level; ++l) w *= 1.0 - changeover_k(r, rho_of(k.rc[l], b, j));
            w *= changeover_k(r, rho_of(k.rc[k.level], b, j));
            const double s = k.G * a.m[j] * w / (r2 * r);
            ax += s * dx;
            ay += s * dy;
            az += s * dz;
        }
#pragma unroll
        for (int d = GL / 2; d > 0; d >>= 1) {
            ax += __shfl_xor(ax, d, GL);
            ay += __shfl_xor(ay, d, GL);
            az += __shfl_xor(az, d, GL);
        }
        if (u == 0) {
            a.vx[b] += k.h * ax;
            a.vy[b] += k.h * ay;
            a.vz[b] += k.h * az;
        }
    }
}

// ---------------------------------------------------------------------------
// Host sequencing
// ---------------------------------------------------------------------------
struct LevelRun {
    genga_bodies *b;
    const genga_params *p;
    const LevelLayout *V;
    char *ws;
    hipStream_t s;

    template <typename T>
    T *at(size_t off) const { return (T *)(ws + off); }
    int32_t *status() const { return (int32_t *)ws; }
    BodyDev bodies_of(int l) const
    {
        BodyDev a;
        a.bodies = at<int32_t>(V->bodies[l]);
        a.nbod = at<int32_t>(V->nbod) + l;
        a.x = b->x; a.y = b->y; a.z = b->z;
        a.vx = b->vx; a.vy = b->vy; a.vz = b->vz;
        a.m = b->m;
        a.status = status();
        return a;
    }
};

static hipError_t build_adj(const LevelRun &R, int l)
{
    const LevelLayout &V = *R.V;
    int32_t *pi = R.at<int32_t>(V.pi[l]), *pj = R.at<int32_t>(V.pj[l]);
    const int64_t *cnt = R.at<int64_t>(V.cnt) + l;
    int32_t *deg = R.at<int32_t>(V.deg[l]), *start = R.at<int32_t>(V.start[l]);
    int32_t *adj = R.at<int32_t>(V.adj[l]), *bod = R.at<int32_t>(V.bodies[l]);
    int32_t *tmp = R.at<int32_t>(V.adj_tmp[l]), *owner = R.at<int32_t>(V.owner[l]);
    int64_t *tsum = R.at<int64_t>(V.tsum);
    const int64_t n = R.b->n;
    const unsigned nt = (unsigned)((n + LT - 1) / LT);
    hipLaunchKernelGGL(k_zero_i32, dim3(LG), dim3(LT), 0, R.s, deg, n);
    hipLaunchKernelGGL(k_adj_count, dim3(LG), dim3(LT), 0, R.s, pi, pj, cnt, V.cap, deg);
    hipLaunchKernelGGL(k_adj_tiles, dim3(nt), dim3(LT), 0, R.s, deg, n, tsum);
    hipLaunchKernelGGL(k_adj_top, dim3(1), dim3(ST), 0, R.s, tsum, (int64_t)nt, start, n,
                       R.at<int32_t>(V.nbod) + l);
    hipLaunchKernelGGL(k_adj_write, dim3(nt), dim3(LT), 0, R.s, deg, n, tsum, start, bod);
    hipLaunchKernelGGL(k_adj_fill, dim3(LG), dim3(LT), 0, R.s, pi, pj, cnt, V.cap, start, deg, tmp,
                       owner);
    hipLaunchKernelGGL(k_adj_rank, dim3(LG), dim3(LT), 0, R.s, start, n, tmp, owner, adj);
    return hipGetLastError();
}

static hipError_t level_kick(const LevelRun &R, int l, double h)
{
    const LevelLayout &V = *R.V;
    LevelKickDev k;
    k.a = R.bodies_of(l - 1);
    k.start = R.at<int32_t>(V.start[l - 1]);
    k.adj = R.at<int32_t>(V.adj[l - 1]);
    for (int q = 0; q < GENGA_MAX_LEVELS; ++q) k.rc[q] = nullptr;
    k.rc[0] = R.b->rc;
    for (int q = 1; q <= l; ++q) k.rc[q] = R.at<double>(V.rc[q]);
    k.level = l;
    k.G = R.p->G;
    k.h = h;
    hipLaunchKernelGGL(k_level_kick, dim3(LG), dim3(LT), 0, R.s, k);
    return hipGetLastError();
}

// Level l >= 1 over list l - 1, sub-steps of dt_l.
static hipError_t advance(const LevelRun &R, int l, double dt_l)
{
    const LevelLayout &V = *R.V;
    const genga_params *p = R.p;
    const int64_t n = R.b->n;
    const bool deeper = l < V.L - 1;
    hipError_t e;
    for (int sub = 0; sub < p->substeps; ++sub) {
        BodyDev up = R.bodies_of(l - 1);
        hipLaunchKernelGGL(k_rcrit_list, dim3(LG), dim3(LT), 0, R.s, up, R.at<double>(V.rc[l]),
                           p->m_star, dt_l, p->n1, p->n2);
        DetectDev d;
        d.in_i = R.at<int32_t>(V.pi[l - 1]);
        d.in_j = R.at<int32_t>(V.pj[l - 1]);
        d.in_cnt = R.at<int64_t>(V.cnt) + (l - 1);
        d.out_i = R.at<int32_t>(V.pi[l]);
        d.out_j = R.at<int32_t>(V.pj[l]);
        d.out_cnt = R.at<int64_t>(V.cnt) + l;
        d.lcount = R.at<int64_t>(V.lcount) + l;
        d.cap = V.cap;
        d.x = R.b->x; d.y = R.b->y; d.z = R.b->z;
        d.rc = R.at<double>(V.rc[l]);
        d.bcnt = R.at<int64_t>(V.bcnt);
        hipLaunchKernelGGL(k_detect_count, dim3(DB), dim3(LT), 0, R.s, d);
        hipLaunchKernelGGL(k_detect_scan, dim3(1), dim3(DB), 0, R.s, d);
        hipLaunchKernelGGL(k_detect_write, dim3(DB), dim3(LT), 0, R.s, d);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = level_kick(R, l, 0.5 * dt_l)) != hipSuccess) return e;
        if (deeper) {
            if ((e = build_adj(R, l)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, R.s, R.bodies_of(l),
                               R.at<double>(V.shadow[l]), n, 1);
        }
        hipLaunchKernelGGL(k_drift_list, dim3(LG), dim3(LT), 0, R.s, up, p->G * p->m_star, dt_l);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (deeper) {
            hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, R.s, R.bodies_of(l),
                               R.at<double>(V.shadow[l]), n, 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = advance(R, l + 1, dt_l / p->substeps)) != hipSuccess) return e;
        }
        if ((e = level_kick(R, l, 0.5 * dt_l)) != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

LevelLayout make_level_layout(int64_t n, const genga_params *p, size_t base)
{
    LevelLayout V;
    if (!p || p->slevels < 2) {
        V.total = base;
        return V;
    }
    V.L = p->slevels;
    V.cap = p->level_capacity;
    size_t off = align_up(base);
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    V.lcount = take(sizeof(int64_t) * V.L);
    V.cnt = take(sizeof(int64_t) * V.L);
    V.nbod = take(sizeof(int32_t) * V.L);
    V.bcnt = take(sizeof(int64_t) * DB);
    V.tsum = take(sizeof(int64_t) * 2 * (size_t)((n + LT - 1) / LT));
    for (int l = 0; l < V.L; ++l) {
        V.pi[l] = take(sizeof(int32_t) * (size_t)V.cap);
        V.pj[l] = take(sizeof(int32_t) * (size_t)V.cap);
        if (l >= 1) V.rc[l] = take(sizeof(double) * (size_t)n);
        if (l < V.L - 1) {
            V.start[l] = take(sizeof(int32_t) * (size_t)(n + 1));
            V.adj[l] = take(sizeof(int32_t) * 2 * (size_t)V.cap);
            V.adj_tmp[l] = take(sizeof(int32_t) * 2 * (size_t)V.cap);
            V.owner[l] = take(sizeof(int32_t) * 2 * (size_t)V.cap);
            V.deg[l] = take(sizeof(int32_t) * (size_t)n);
            V.bodies[l] = take(sizeof(int32_t) * (size_t)n);
            V.shadow[l] = take(sizeof(double) * 6 * (size_t)n);
        }
    }
    V.total = off;
    return V;
}

genga_pairs level0_pairs(const LevelLayout &V, char *ws)
{
    genga_pairs q;
    q.i = (int32_t *)(ws + V.pi[0]);
    q.j = (int32_t *)(ws + V.pj[0]);
    q.capacity = V.cap;
    q.count = (int64_t *)(ws + V.cnt);
    return q;
}

hipError_t levels_before_drift(const genga_bodies *b, const LevelLayout &V, genga_pairs *out,
                               char *ws, hipStream_t s)
{
    LevelRun R{const_cast<genga_bodies *>(b), nullptr, &V, ws, s};
    const int64_t *cnt0 = R.at<int64_t>(V.cnt);
    hipLaunchKernelGGL(k_level_begin, dim3(1), dim3(64), 0, s, R.at<int64_t>(V.lcount), V.L, cnt0);
    if (out) {
        hipLaunchKernelGGL(k_copy_pairs, dim3(LG), dim3(LT), 0, s, R.at<int32_t>(V.pi[0]),
                           R.at<int32_t>(V.pj[0]), cnt0, V.cap, out->i, out->j, out->capacity,
                           out->count, R.status());
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = build_adj(R, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, s, R.bodies_of(0),
                       R.at<double>(V.shadow[0]), b->n, 1);
    return hipGetLastError();
}

hipError_t levels_after_drift(genga_bodies *b, const genga_params *p, const LevelLayout &V,
                              char *ws, hipStream_t s)
{
    LevelRun R{b, p, &V, ws, s};
    hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, s, R.bodies_of(0),
                       R.at<double>(V.shadow[0]), b->n, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return advance(R, 1, p->dt / p->substeps);
}

}  // namespace genga
