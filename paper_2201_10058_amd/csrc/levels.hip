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
#include <algorithm>
#include <climits>
#include <mutex>

#include "device_common.h"
#include "genga_internal.h"
#include "kepler.h"

namespace genga {

namespace {

constexpr int LT = 256;     // threads per block of the list kernels
constexpr int LG = 1024;    // blocks of the grid-stride list kernels
constexpr int LG_BIG = 512; // workgroups of the Bulirsch-Stoer class of 9-512 bodies (2 per CU)
constexpr int GROUP_BLOCK = 512;   // largest group of the one-workgroup class
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

__global__ __launch_bounds__(64) void k_level_begin(int64_t *lcount, int L, const int64_t *cnt0,
                                                    int64_t *gstats, int64_t *coll_count)
{
    const int t = threadIdx.x;
    if (t < L) lcount[t] = t == 0 ? *cnt0 : 0;
    if (gstats && t < 2) gstats[t] = 0;
    if (coll_count && t == 0) *coll_count = 0;
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
// Close-encounter groups of a list: connected components of its pair graph
// by a lock-free union-find (a root is hooked under the smaller root, so each
// group's root is its smallest body, whatever the order of the unions), then
// per-root sizes, a scan over the roots in ascending order, and the members
// of each group placed in ascending order (rank among the group's members).
// ---------------------------------------------------------------------------
// A parent read through the caches (workgroup scope) may be an older value:
// every value a body's parent ever held is still one of its ancestors (trees
// only merge) and a root's parent was itself until it was hooked, so an old
// value only makes a walk stop early, at a node that was a root; the hook's
// exchange then fails and returns the current parent.  (Reads at device
// scope, from memory, made the 65,536-body ring's unions 1.5 ms.)
__device__ __forceinline__ int32_t uf_load(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x, halving the path on the way: a non-root's parent may be
// replaced by any of its ancestors (parents only point to smaller bodies and
// a non-root never becomes a root again), so plain atomic stores of the
// grandparent are safe under concurrent hooks and keep the chains short (a
// ring's chain is as long as the ring otherwise).
__device__ __forceinline__ int32_t uf_find(int32_t *parent, int32_t x)
{
    for (;;) {
        const int32_t p = uf_load(parent + x);
        if (p == x) return x;
        const int32_t gp = uf_load(parent + p);
        if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

// atomicAdd(ctr + key, 1) for every active lane, one atomic per distinct key
// of the wave; returns the lane's slot (the old value plus its rank among
// the wave's lanes with the same key).
__device__ __forceinline__ int32_t wave_add_by_key(int32_t *ctr, int32_t key, bool active)
{
    unsigned long long todo = __ballot(active);
    int32_t slot = 0;
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int32_t k = __shfl(key, lead, 64);
        const unsigned long long same = __ballot(active && key == k);
        int32_t base = 0;
        if ((int)(threadIdx.x & 63) == lead) base = atomicAdd(ctr + k, __popcll(same));
        base = __shfl(base, lead, 64);
        if (active && key == k) {
            const unsigned long long lower = same & ((1ull << (threadIdx.x & 63)) - 1ull);
            slot = base + __popcll(lower);
        }
        todo &= ~same;
    }
    return slot;
}

__global__ __launch_bounds__(LT) void k_group_init(int32_t *parent, int32_t *flag, int32_t *gsize,
                                                   int32_t *gfill, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * LT + threadIdx.x; k < n; k += (int64_t)gridDim.x * LT) {
        parent[k] = (int32_t)k;
        flag[k] = 0;
        gsize[k] = 0;
        gfill[k] = 0;
    }
}

__global__ __launch_bounds__(LT) void k_group_union(const int32_t *pi, const int32_t *pj,
                                                    const int64_t *cnt, int64_t cap,
                                                    int32_t *parent, int32_t *flag)
{
    const int64_t m = list_len(cnt, cap);
    for (int64_t p = (int64_t)blockIdx.x * LT + threadIdx.x; p < m; p += (int64_t)gridDim.x * LT) {
        const int32_t i = pi[p], j = pj[p];
        flag[i] = 1;
        flag[j] = 1;
        int32_t a0 = i, b0 = j;
        for (;;) {
            int32_t ra = uf_find(parent, a0), rb = uf_find(parent, b0);
            if (ra == rb) break;   // a common ancestor: one tree
            if (ra < rb) {
                const int32_t t = ra;
                ra = rb;
                rb = t;
            }
            // hook the larger root under the smaller (a root is the smallest
            // body of its tree, so rb < ra lies in another tree); a failed
            // exchange means ra was hooked meanwhile: go on from its current
            // parent, which the exchange returns
            const int32_t old = atomicCAS(parent + ra, ra, rb);
            if (old == ra) break;
            a0 = old;
            b0 = rb;
        }
    }
}

// Root of every listed body (into lab), members counted per root.
__global__ __launch_bounds__(LT) void k_group_root(int32_t *parent, const int32_t *flag,
                                                   int32_t *lab, int32_t *gsize, int64_t n)
{
    for (int64_t k0 = (int64_t)blockIdx.x * LT; k0 < n; k0 += (int64_t)gridDim.x * LT) {
        const int64_t k = k0 + threadIdx.x;
        const bool on = k < n && flag[k];
        int32_t r = 0;
        if (on) {
            r = uf_find(parent, (int32_t)k);
            lab[k] = r;
        }
        wave_add_by_key(gsize, r, on);
    }
}

// Tile sums of (members of the groups whose root is in the tile, roots).
__global__ __launch_bounds__(LT) void k_group_tiles(const int32_t *flag, const int32_t *lab,
                                                    const int32_t *gsize, int64_t n, int64_t *tsum)
{
    __shared__ int64_t sm[LT / 64];
    const int64_t k = (int64_t)blockIdx.x * LT + threadIdx.x;
    const bool root = k < n && flag[k] && lab[k] == k;
    int64_t tm, tr;
    block_excl_scan<LT>(root ? gsize[k] : 0, &tm, sm);
    block_excl_scan<LT>(root ? 1 : 0, &tr, sm);
    if (threadIdx.x == 0) {
        tsum[2 * blockIdx.x] = tm;
        tsum[2 * blockIdx.x + 1] = tr;
    }
}

__global__ __launch_bounds__(ST) void k_group_top(int64_t *tsum, int64_t ntiles, int32_t *gcount,
                                                  int32_t *big, unsigned long long *gsync)
{
    __shared__ int64_t sm[ST / 64];
    const int t = threadIdx.x;
    const int64_t ch = (ntiles + ST - 1) / ST;
    const int64_t k0 = min(ntiles, t * ch), k1 = min(ntiles, k0 + ch);
    int64_t sa = 0, sb = 0;
    for (int64_t k = k0; k < k1; ++k) {
        sa += tsum[2 * k];
        sb += tsum[2 * k + 1];
    }
    int64_t ta, tb;
    int64_t oa = block_excl_scan<ST>(sa, &ta, sm);
    int64_t ob = block_excl_scan<ST>(sb, &tb, sm);
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t a = tsum[2 * k], b = tsum[2 * k + 1];
        tsum[2 * k] = oa;
        tsum[2 * k + 1] = ob;
        oa += a;
        ob += b;
    }
    if (t == 0) {
        gcount[0] = (int32_t)tb;   // groups
        gcount[1] = (int32_t)ta;   // members
        if (big) {
            // the grid solver's list and barrier state, fresh for its launch:
            // arrivals, abort flag, three maximum slots, three minimum slots
            big[0] = 0;
            for (int k = 0; k < 5; ++k) gsync[k] = 0;
            for (int k = 5; k < 8; ++k) gsync[k] = (unsigned long long)LLONG_MAX;
        }
    }
}

__global__ __launch_bounds__(LT) void k_group_write(const int32_t *flag, const int32_t *lab,
                                                    const int32_t *gsize, int64_t n,
                                                    const int64_t *tsum, int32_t *gstart,
                                                    int32_t *groot, int32_t *big)
{
    __shared__ int64_t sm[LT / 64];
    const int64_t k = (int64_t)blockIdx.x * LT + threadIdx.x;
    const bool root = k < n && flag[k] && lab[k] == k;
    int64_t tm, tr;
    const int64_t om = block_excl_scan<LT>(root ? gsize[k] : 0, &tm, sm);
    const int64_t orr = block_excl_scan<LT>(root ? 1 : 0, &tr, sm);
    if (root) {
        gstart[k] = (int32_t)(tsum[2 * blockIdx.x] + om);
        groot[tsum[2 * blockIdx.x + 1] + orr] = (int32_t)k;
        // groups beyond one workgroup, for the grid solver (any order)
        if (big && gsize[k] > GROUP_BLOCK) big[1 + atomicAdd(big, 1)] = (int32_t)k;
    }
}

__global__ __launch_bounds__(LT) void k_group_fill(const int32_t *flag, const int32_t *lab,
                                                   const int32_t *gstart, int32_t *gfill,
                                                   int32_t *gtmp, int64_t n)
{
    for (int64_t k0 = (int64_t)blockIdx.x * LT; k0 < n; k0 += (int64_t)gridDim.x * LT) {
        const int64_t k = k0 + threadIdx.x;
        const bool on = k < n && flag[k];
        const int32_t r = on ? lab[k] : 0;
        const int32_t slot = wave_add_by_key(gfill, r, on);
        if (on) gtmp[gstart[r] + slot] = (int32_t)k;
    }
}

__global__ __launch_bounds__(LT) void k_group_rank(const int32_t *lab, const int32_t *gstart,
                                                   const int32_t *gsize, const int32_t *gtmp,
                                                   const int32_t *gcount, int32_t *gmem)
{
    const int64_t total = gcount[1];
    for (int64_t e = (int64_t)blockIdx.x * LT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * LT) {
        const int32_t k = gtmp[e], r = lab[k];
        const int32_t s0 = gstart[r], g = gsize[r];
        // the grid solver orders a large group's members itself (by cell,
        // then body): its slots keep the arrival order, sparing the
        // quadratic ranking
        if (g > GROUP_BLOCK) {
            gmem[e] = k;
            continue;
        }
        int32_t rank = 0;
        for (int32_t q = s0; q < s0 + g; ++q) rank += gtmp[q] < k;
        gmem[s0 + rank] = k;
    }
}

// ---------------------------------------------------------------------------
// Direct solver: one thread per member; groups of up to 8 bodies take 8 lanes
// of a wave each, larger ones a workgroup of 512 threads (Table 1 splits them
// into more classes up to 512 bodies; here they are rare, and 512 threads
// hold the extrapolation tableau in registers at 2 waves per SIMD with 68 KB
// of LDS).  The
// group's flow (Kepler force of the star plus the remainder R of the mutual
// forces) is integrated over H by Bulirsch-Stoer steps: the modified
// midpoint rule with n = 2, 4, ..., 2 KM sub-steps, polynomial extrapolation
// in (h/n)^2 (Neville), a step accepted when the last two extrapolations
// agree within eps (relative to each member's position and velocity
// magnitudes), else retried with half the step; after a step that converged
// early the next one doubles (never beyond what is left of H).
// ---------------------------------------------------------------------------
constexpr int KM = 8;
constexpr int BS_TRIES = 4096;

struct BsDev {
    const int32_t *groot, *gstart, *gsize, *gmem, *gcount;
    const double *shadow;               // [6][n] state before the drift
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz;
    double *m;                          // written by mergers
    const double *rc[GENGA_MAX_LEVELS]; // levels 0 .. nlev - 1 weigh R
    int nlev;
    double G, mu, H, eps;
    int32_t *status;
    unsigned long long *gstats;         // groups, largest group
    // collisions (radius non-null): radii (written by mergers), contact
    // tolerance, records (survivor, absorbed, lost energy)
    double *radius;
    double coll_tol;
    int32_t *coll_i, *coll_j;
    double *coll_du;
    unsigned long long *coll_count;
    int64_t coll_cap;
};

// 1/sqrt(x) and 1/x from the hardware estimates (v_rsq_f64, v_rcp_f64) and two
// Newton steps each: the serial chain of the group derivative is dominated
// by latency, and these are several times shorter than the IEEE square root
// and division; two steps take the estimates' 2^-24-level error below the
// binary64 rounding level, far inside the Bulirsch-Stoer tolerance.
__device__ __forceinline__ double rsq2(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-x, y * y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-x, y * y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}

__device__ __forceinline__ double rcp2(double x)
{
    double t = __builtin_amdgcn_rcp(x);
    t = __builtin_fma(t, __builtin_fma(-x, t, 1.0), t);
    return __builtin_fma(t, __builtin_fma(-x, t, 1.0), t);
}

// R = prod_l (1 - K(r; rho_l)) with y_l = r / (0.9 rho_l) - 1/9, from
// irho_l = 1 / rho_l = min(1 / rc_i, 1 / rc_j).  The members' reciprocal
// critical radii are formed once per group (the radii do not change during
// the integration) and read from LDS: level l of member i at ia[l * sa], of
// member j at ib[l * sb].
__device__ __forceinline__ double bs_remainder(double r, const double *ia, int sa, const double *ib,
                                               int sb, int nlev)
{
    double R = 1.0;
    for (int l = 0; l < nlev; ++l) {
        const double xa = ia[l * sa], xb = ib[l * sb];
        const double irho = xa < xb ? xa : xb;
        const double yv = __builtin_fma(r * irho, 10.0 / 9.0, -1.0 / 9.0);
        R *= 1.0 - changeover_of_y(yv);
    }
    return R;
}

__device__ __forceinline__ double wave_min_all(double v)
{
    for (int d = 32; d > 0; d >>= 1) {
        const double o = __shfl_xor(v, d, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ double wave_max_all(double v)
{
    for (int d = 32; d > 0; d >>= 1) {
        const double o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Squared gap between the box (lo, hi) and the box B = (lo, hi) of another
// tile: a lower bound of the squared distance of any two of their members.
__device__ __forceinline__ double box_gap2(const double lo[3], const double hi[3], const double *B)
{
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double a1 = B[c] - hi[c], a2 = lo[c] - B[3 + c];
        const double gc = a1 > a2 ? a1 : a2;
        d2 += gc > 0.0 ? gc * gc : 0.0;
    }
    return d2;
}

template <int BT>
struct BsSmem {
    double px[BT], py[BT], pz[BT], m[BT];
    double pv[3][BT], R[BT];
    double rcd[BT];                     // deepest-level rc
    double box[BT / 64][8];             // each wave's box of its members' positions
    double trho[BT / 64];               // each wave's largest deepest-level rc
    int32_t idx[BT];
    double irc[GENGA_MAX_LEVELS][BT];   // 1 / rc of each level
    double red[BT / 64];
    long long ired[BT / 64];
};

// Partner sum of member t at its position (o) from the positions in LDS,
// over share `sub` of S: the partners q = sub, sub + S, ... of every partner
// wave that is not skipped.  The partners come by waves of 64: a wave whose
// box stays beyond the larger deepest-level critical radius of the two waves
// from the own wave's box holds no partner with R > 0 and is skipped (its
// terms are exact zeros), as is each single partner beyond that radius.
template <int BT>
__device__ __forceinline__ void bs_accel(const BsDev &a, const BsSmem<BT> &sm, int t, int g,
                                         int S, int sub, const double o[3], double acc[3])
{
    const double *BI = sm.box[t >> 6];
    const double lo[3] = {BI[0], BI[1], BI[2]}, hi[3] = {BI[3], BI[4], BI[5]};
    const int nw = (g + 63) >> 6;
    const double rhoI = sm.trho[t >> 6];
    for (int J = 0; J < nw; ++J) {
        const double rr = rhoI > sm.trho[J] ? rhoI : sm.trho[J];
        if (box_gap2(lo, hi, sm.box[J]) > rr * rr * (1.0 + 0x1p-18)) continue;
        const int q1 = g < J * 64 + 64 ? g : J * 64 + 64;
        for (int q = J * 64 + sub; q < q1; q += S) {
            if (q == t) continue;
            const double dx = sm.px[q] - o[0], dy = sm.py[q] - o[1], dz = sm.pz[q] - o[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            // beyond the larger deepest-level radius R = 0 exactly: the term
            // is an exact zero and skipping it leaves the sum unchanged
            const double rq = sm.rcd[t] > sm.rcd[q] ? sm.rcd[t] : sm.rcd[q];
            if (r2 > rq * rq * (1.0 + 0x1p-18)) continue;
            const double ir = rsq2(r2);
            const double R = bs_remainder(r2 * ir, &sm.irc[0][t], BT, &sm.irc[0][q], BT, a.nlev);
            const double s = a.G * sm.m[q] * R * (ir * ir * ir);
            acc[0] += s * dx;
            acc[1] += s * dy;
            acc[2] += s * dz;
        }
    }
}

// Publish positions (and each wave's box), then every member's derivative
// at them: the star's pull plus the S shares' partner sums, added in share
// order (the waves of a share hold copies of the same members; only share 0
// writes).  The shares' sums pass through pv, which no evaluation uses.
template <int BT>
__device__ __forceinline__ void bs_deriv(const BsDev &a, BsSmem<BT> &sm, int t, int g, int S,
                                         int sub, const double z[6], double f[6])
{
    __syncthreads();   // the previous evaluation has finished reading
    const bool mem = t < g, own = mem && sub == 0;
    if (own) {
        sm.px[t] = z[0];
        sm.py[t] = z[1];
        sm.pz[t] = z[2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double lo = wave_min_all(mem ? z[c] : INFINITY);
        const double hi = wave_max_all(mem ? z[c] : -INFINITY);
        if ((threadIdx.x & 63) == 0 && own) {
            sm.box[t >> 6][c] = lo;
            sm.box[t >> 6][3 + c] = hi;
        }
    }
    __syncthreads();
    f[0] = z[3];
    f[1] = z[4];
    f[2] = z[5];
    double p[3] = {0.0, 0.0, 0.0};
    if (mem) bs_accel<BT>(a, sm, t, g, S, sub, z, p);
    double k[3] = {0.0, 0.0, 0.0};
    if (mem) {
        const double r2s = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
        const double irs = rsq2(r2s);
        const double ks = -a.mu * (irs * irs * irs);
        k[0] = ks * z[0];
        k[1] = ks * z[1];
        k[2] = ks * z[2];
    }
    if (S > 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sm.pv[c][threadIdx.x] = p[c];
        __syncthreads();
        const int w0 = (threadIdx.x >> 6) - sub, lane = threadIdx.x & 63;
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) k[c] += sm.pv[c][(w0 + s) * 64 + lane];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) k[c] += p[c];
    }
    f[3] = k[0];
    f[4] = k[1];
    f[5] = k[2];
}

template <int BT>
__device__ __forceinline__ double bs_block_max(BsSmem<BT> &sm, double v)
{
    for (int d = 32; d > 0; d >>= 1) {
        const double o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sm.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sm.red[0];
#pragma unroll
    for (int w = 1; w < BT / 64; ++w) r = sm.red[w] > r ? sm.red[w] : r;
    return r;
}

// How the members of a group see each other: a workgroup with the positions
// in LDS (BlockPol), or GS lanes of one wave exchanging them by shuffles
// (LanePol, several small groups per wave and no barriers).
// Both policies also expose, for the collision search and the merger: the
// whole state of member q after publish(), its mass, radius and body index,
// a group-wide minimum of an integer key, and updates of the own member's
// mass and radius.
template <int BT>
struct BlockPol {
    BsSmem<BT> &sm;
    int t, g;
    int S, sub;   // waves per member (the group's shares), this wave's share
    __device__ void deriv(const BsDev &a, const double z[6], double f[6])
    {
        bs_deriv<BT>(a, sm, t, g, S, sub, z, f);
    }
    __device__ double gmax(double v) { return bs_block_max<BT>(sm, v); }
    __device__ bool member() const { return t < g; }
    __device__ bool owner() const { return t < g && sub == 0; }
    __device__ int self() const { return t; }
    __device__ long long overlap(const BsDev &a, const double z[6]);
    __device__ void publish(const double z[6])
    {
        __syncthreads();
        if (owner()) {
            sm.px[t] = z[0];
            sm.py[t] = z[1];
            sm.pz[t] = z[2];
            sm.pv[0][t] = z[3];
            sm.pv[1][t] = z[4];
            sm.pv[2][t] = z[5];
        }
        __syncthreads();
    }
    __device__ void get(int q, double o[6]) const
    {
        o[0] = sm.px[q];
        o[1] = sm.py[q];
        o[2] = sm.pz[q];
        o[3] = sm.pv[0][q];
        o[4] = sm.pv[1][q];
        o[5] = sm.pv[2][q];
    }
    __device__ double mass(int q) const { return sm.m[q]; }
    __device__ double rad(int q) const { return sm.R[q]; }
    __device__ int idx(int q) const { return sm.idx[q]; }
    __device__ void set_own(double m, double R)
    {
        if (owner()) {
            sm.m[t] = m;
            sm.R[t] = R;
        }
    }
    __device__ long long gmin(long long v)
    {
        for (int d = 32; d > 0; d >>= 1) {
            const long long o = __shfl_xor(v, d, 64);
            v = o < v ? o : v;
        }
        __syncthreads();
        if ((threadIdx.x & 63) == 0) sm.ired[threadIdx.x >> 6] = v;
        __syncthreads();
        long long r = sm.ired[0];
#pragma unroll
        for (int w = 1; w < BT / 64; ++w) r = sm.ired[w] < r ? sm.ired[w] : r;
        return r;
    }
};

template <int GS>
struct LanePol {
    int u, g;
    double m, R;
    int32_t bidx;
    double zc[6];
    const double *irc;   // 1 / rc of each level: LDS, level l at irc[l * LT]; lane q at + q - u
    __device__ bool member() const { return u < g; }
    __device__ bool owner() const { return true; }
    __device__ int self() const { return u; }
    __device__ long long overlap(const BsDev &a, const double z[6]);
    __device__ void publish(const double z[6])
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) zc[c] = z[c];
    }
    __device__ void get(int q, double o[6]) const
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = __shfl(zc[c], q, GS);
    }
    __device__ double mass(int q) const { return __shfl(m, q, GS); }
    __device__ double rad(int q) const { return __shfl(R, q, GS); }
    __device__ int idx(int q) const { return __shfl(bidx, q, GS); }
    __device__ void set_own(double mm, double RR)
    {
        if (u < g) {
            m = mm;
            R = RR;
        }
    }
    __device__ long long gmin(long long v)
    {
        for (int d = GS / 2; d > 0; d >>= 1) {
            const long long o = __shfl_xor(v, d, GS);
            v = o < v ? o : v;
        }
        return v;
    }
    // every lane of the group runs the same partner loop (the shuffles need
    // all GS lanes); only members add terms
    __device__ void deriv(const BsDev &a, const double z[6], double f[6])
    {
        f[0] = z[3];
        f[1] = z[4];
        f[2] = z[5];
        double acc[3] = {0.0, 0.0, 0.0};
        const bool mem = u < g;
        if (mem) {
            const double r2s = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
            const double irs = rsq2(r2s);
            const double ks = -a.mu * (irs * irs * irs);
            acc[0] = ks * z[0];
            acc[1] = ks * z[1];
            acc[2] = ks * z[2];
        }
        for (int q = 0; q < g; ++q) {
            const double xq = __shfl(z[0], q, GS), yq = __shfl(z[1], q, GS),
                         zq = __shfl(z[2], q, GS), mq = __shfl(m, q, GS);
            if (!mem || q == u) continue;
            const double dx = xq - z[0], dy = yq - z[1], dz = zq - z[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = rsq2(r2);
            const double R = bs_remainder(r2 * ir, irc, LT, irc + (q - u), LT, a.nlev);
            const double s = a.G * mq * R * (ir * ir * ir);
            acc[0] += s * dx;
            acc[1] += s * dy;
            acc[2] += s * dz;
        }
        f[3] = acc[0];
        f[4] = acc[1];
        f[5] = acc[2];
    }
    __device__ double gmax(double v)
    {
        for (int d = GS / 2; d > 0; d >>= 1) {
            const double o = __shfl_xor(v, d, GS);
            v = o > v ? o : v;
        }
        return v;
    }
};

// One Bulirsch-Stoer step of length h from y: the modified midpoint rule
// with n = 2, 4, ..., 2 KM sub-steps and Neville's extrapolation (the tableau
// updated in place, the loop over the sequence unrolled so that it stays in
// registers).  Returns the number of extrapolations that met the tolerance
// (-1 if none did; yout then holds the last one).
template <class Pol>
__device__ int bs_step(const BsDev &a, Pol &P, const double y[6], double h, double yout[6])
{
    double f0[6];
    P.deriv(a, y, f0);
    const double sx = __builtin_sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]) +
                      h * __builtin_sqrt(f0[0] * f0[0] + f0[1] * f0[1] + f0[2] * f0[2]);
    const double sv = __builtin_sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]) +
                      h * __builtin_sqrt(f0[3] * f0[3] + f0[4] * f0[4] + f0[5] * f0[5]);
    double T[KM][6];
    int kdone = -1;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int nk = 2 * (k + 1);
        const double hh = h / nk;
        double z0[6], z1[6], fz[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            z0[c] = y[c];
            z1[c] = y[c] + hh * f0[c];
        }
#pragma unroll 1
        for (int q = 1; q < nk; ++q) {
            P.deriv(a, z1, fz);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double z2 = z0[c] + 2.0 * hh * fz[c];
                z0[c] = z1[c];
                z1[c] = z2;
            }
        }
        P.deriv(a, z1, fz);
        // row k of the tableau: T[0] = the midpoint result, T[j] from T[j - 1]
        // (this row) and the previous row's T[j - 1]
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double old = T[0][c];
            T[0][c] = 0.5 * (z0[c] + z1[c] + hh * fz[c]);
#pragma unroll
            for (int j = 1; j <= k; ++j) {
                const double ratio = (double)nk / (double)(nk - 2 * j);
                const double den = ratio * ratio - 1.0;
                const double oj = T[j][c];
                T[j][c] = T[j - 1][c] + (T[j - 1][c] - old) / den;
                old = oj;
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) yout[c] = T[k][c];
        if (k > 0) {
            double err = 0.0;
            if (P.member()) {
                double ex = 0.0, ev = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double dxc = fabs(T[k][c] - T[k - 1][c]);
                    const double dvc = fabs(T[k][c + 3] - T[k - 1][c + 3]);
                    // (written so that a NaN propagates into the error)
                    ex = (dxc > ex || dxc != dxc) ? dxc : ex;
                    ev = (dvc > ev || dvc != dvc) ? dvc : ev;
                }
                const double e1 = ex / (sx + 1e-300), e2 = ev / (sv + 1e-300);
                err = e1 > e2 ? e1 : e2;
                // a step through a singularity (two members passing through
                // each other) yields NaN: count it as not converged, so that
                // every member takes the same decision
                if (!(err <= INFINITY)) err = INFINITY;
            }
            err = P.gmax(err);
            if (err <= a.eps) {
                kdone = k;
                break;
            }
        }
    }
    return kdone;
}

// The first overlapping pair of the group at state z (a < b, encoded as
// a * KEY_BASE + b), or NO_PAIR.  Uniform over the group.
constexpr long long KEY_BASE = 65536;
constexpr long long NO_PAIR = LLONG_MAX;

template <class Pol>
__device__ long long bs_overlap(const BsDev &a, Pol &P, const double z[6])
{
    P.publish(z);
    long long key = NO_PAIR;
    const int u = P.self();
    const double ru = P.rad(u);
    for (int q = 0; q < P.g; ++q) {
        double o[6];
        P.get(q, o);
        const double rq = P.rad(q);
        if (!P.member() || q <= u) continue;
        const double rs = ru + rq;
        const double dx = o[0] - z[0], dy = o[1] - z[1], dz = o[2] - z[2];
        if (rs > 0.0 && dx * dx + dy * dy + dz * dz < rs * rs && key == NO_PAIR)
            key = (long long)u * KEY_BASE + q;
    }
    return P.gmin(key);
}

template <int BT>
__device__ long long BlockPol<BT>::overlap(const BsDev &a, const double z[6])
{
    return bs_overlap(a, *this, z);
}

template <int GS>
__device__ long long LanePol<GS>::overlap(const BsDev &a, const double z[6])
{
    return bs_overlap(a, *this, z);
}

// Distance of members ma, mb at state z (uniform).
template <class Pol>
__device__ double bs_sep(Pol &P, const double z[6], int ma, int mb)
{
    P.publish(z);
    double oa[6], ob[6];
    P.get(ma, oa);
    P.get(mb, ob);
    const double dx = ob[0] - oa[0], dy = ob[1] - oa[1], dz = ob[2] - oa[2];
    return __builtin_sqrt(dx * dx + dy * dy + dz * dz);
}

// Perfect merger of members ma, mb at state z (in place): the survivor (the
// more massive, the lower body index for equal masses) takes the mass-weighted
// position and velocity, the summed mass and the radius (R_a^3 + R_b^3)^(1/3);
// the absorbed body becomes a massless, sizeless ghost at rest at
// (1e6 + index, 0, 0); one record (survivor, absorbed, lost energy
// 1/2 m_a m_b / (m_a + m_b) |v_a - v_b|^2 - G m_a m_b / r).
template <class Pol>
__device__ void bs_merge(const BsDev &a, Pol &P, double z[6], int ma, int mb)
{
    P.publish(z);
    double ya[6], yb[6];
    P.get(ma, ya);
    P.get(mb, yb);
    const double m1 = P.mass(ma), m2 = P.mass(mb), R1 = P.rad(ma), R2 = P.rad(mb);
    const int i1 = P.idx(ma), i2 = P.idx(mb);
    const bool first = m1 > m2 || (m1 == m2 && i1 < i2);
    const int ms = first ? ma : mb, mg = first ? mb : ma;
    const double M = m1 + m2;
    const int u = P.self();
    if (u == ms) {
#pragma unroll
        for (int c = 0; c < 6; ++c) z[c] = (m1 * ya[c] + m2 * yb[c]) / M;
        P.set_own(M, cbrt(R1 * R1 * R1 + R2 * R2 * R2));
        double dv2 = 0.0, dx2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            dx2 += (ya[c] - yb[c]) * (ya[c] - yb[c]);
            dv2 += (ya[c + 3] - yb[c + 3]) * (ya[c + 3] - yb[c + 3]);
        }
        const double du = 0.5 * m1 * m2 / M * dv2 - a.G * m1 * m2 / __builtin_sqrt(dx2);
        if (P.owner()) {
            const unsigned long long slot = atomicAdd(a.coll_count, 1ull);
            if ((int64_t)slot < a.coll_cap) {
                a.coll_i[slot] = first ? i1 : i2;
                a.coll_j[slot] = first ? i2 : i1;
                a.coll_du[slot] = du;
            }
        }
    } else if (u == mg) {
        z[0] = 1e6 + (double)(first ? i2 : i1);
        z[1] = z[2] = z[3] = z[4] = z[5] = 0.0;
        P.set_own(0.0, 0.0);
    }
}

// One group's flow over H from y (in place); returns true if it failed.
// With radii, each accepted step is searched for an overlapping pair; the
// contact is bisected on the step length until the overlap is below
// coll_tol of R_a + R_b, the pair merges there, and the flow continues from
// that time.
template <class Pol>
__device__ bool bs_run(const BsDev &a, Pol &P, double y[6])
{
    double tt = 0.0, h = a.H;
    int tries = 0;
    while (tt < a.H) {      // uniform over the group: every member holds the same tt, h
        const bool last = h >= a.H - tt;
        if (last) h = a.H - tt;
        double yn[6];
        const int kdone = bs_step(a, P, y, h, yn);
        if (kdone >= 0) {
            const long long key = a.radius ? P.overlap(a, yn) : NO_PAIR;
            if (key != NO_PAIR) {
                const int ma = (int)(key / KEY_BASE), mb = (int)(key % KEY_BASE);
                const double rs = P.rad(ma) + P.rad(mb);
                double lo = 0.0, hi = h;
                double yh[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) yh[c] = yn[c];
                for (int it = 0; it < 60; ++it) {
                    if ((rs - bs_sep(P, yh, ma, mb)) / rs < a.coll_tol) break;
                    const double mid = 0.5 * (lo + hi);
                    double ym[6];
                    bs_step(a, P, y, mid, ym);
                    if (bs_sep(P, ym, ma, mb) < rs) {
                        hi = mid;
#pragma unroll
                        for (int c = 0; c < 6; ++c) yh[c] = ym[c];
                    } else {
                        lo = mid;
                    }
                }
                bs_merge(a, P, yh, ma, mb);
#pragma unroll
                for (int c = 0; c < 6; ++c) y[c] = yh[c];
                tt = (last && hi == h) ? a.H : tt + hi;
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) y[c] = yn[c];
                tt = last ? a.H : tt + h;
                if (kdone < KM / 2) h *= 2.0;
            }
        } else {
            h *= 0.5;
        }
        if (++tries > BS_TRIES || h < a.H * 1e-12) return true;
    }
    return false;
}

__device__ __forceinline__ void bs_store(const BsDev &a, int32_t b, const double y[6])
{
    a.x[b] = y[0];
    a.y[b] = y[1];
    a.z[b] = y[2];
    a.vx[b] = y[3];
    a.vy[b] = y[4];
    a.vz[b] = y[5];
}

// Groups of at most GS bodies, GS lanes each (the many small groups).
constexpr int BS_GS = 8;

template <int GS>
__global__ __launch_bounds__(LT) void k_bs_lanes(BsDev a)
{
    __shared__ double irc_sm[GENGA_MAX_LEVELS][LT];
    const int u = threadIdx.x % GS;
    const int64_t ng = a.gcount[0];
    const int64_t stride = (int64_t)gridDim.x * (LT / GS);
    for (int64_t gi = ((int64_t)blockIdx.x * LT + threadIdx.x) / GS; gi < ng; gi += stride) {
        const int32_t root = a.groot[gi];
        const int g = a.gsize[root];
        if (g > GS) continue;                        // a workgroup class's group
        if (u == 0) {
            atomicAdd(a.gstats, 1ull);
            atomicMax(a.gstats + 1, (unsigned long long)g);
        }
        LanePol<GS> P;
        P.u = u;
        P.g = g;
        P.m = 0.0;
        P.R = 0.0;
        for (int c = 0; c < 6; ++c) P.zc[c] = 0.0;
        P.irc = &irc_sm[0][threadIdx.x];
        const int32_t b = u < g ? a.gmem[a.gstart[root] + u] : 0;
        P.bidx = b;
        double y[6] = {0, 0, 0, 0, 0, 0};
        if (u < g) {
#pragma unroll
            for (int c = 0; c < 6; ++c) y[c] = a.shadow[(size_t)c * a.n + b];
            P.m = a.m[b];
            P.R = a.radius ? a.radius[b] : 0.0;
            for (int l = 0; l < a.nlev; ++l) irc_sm[l][threadIdx.x] = rcp2(a.rc[l][b]);
        }
        const bool failed = bs_run(a, P, y);
        if (failed && u == 0) atomicOr(a.status, ST_NOCONV);
        if (u < g) {
            bs_store(a, b, y);
            if (a.radius) {
                a.m[b] = P.m;
                a.radius[b] = P.R;
            }
        }
    }
}

// Groups of lo < size <= BT, one workgroup each (larger ones are the grid
// solver's).  A group of fewer members than threads spreads each member over
// S waves (S = BT / 64 over the member waves, a power of two): the waves of
// member wave I are I * S ... I * S + S - 1, each taking one share of the
// partners, and the first of them (the owner) alone writes.
template <int BT>
__global__ __launch_bounds__(BT) void k_bs(BsDev a, int lo)
{
    __shared__ BsSmem<BT> sm;
    // (the wave index is uniform: the partner loops then run on scalar registers)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int ng = a.gcount[0];
    for (int gi = blockIdx.x; gi < ng; gi += gridDim.x) {
        const int32_t root = a.groot[gi];
        const int g = a.gsize[root];
        if (g <= lo || g > BT) continue;             // another class's group
        if (threadIdx.x == 0) {
            atomicAdd(a.gstats, 1ull);
            atomicMax(a.gstats + 1, (unsigned long long)g);
        }
        const int nw = (g + 63) >> 6;
        int S = 1;
        while (nw * S * 2 <= BT / 64) S *= 2;
        const int t = (w / S) * 64 + lane, sub = w % S;
        BlockPol<BT> P{sm, t, g, S, sub};
        const int32_t b = t < g ? a.gmem[a.gstart[root] + t] : 0;
        double y[6] = {0, 0, 0, 0, 0, 0};
        double rcd = 0.0;
        if (t < g) {
#pragma unroll
            for (int c = 0; c < 6; ++c) y[c] = a.shadow[(size_t)c * a.n + b];
            rcd = a.rc[a.nlev - 1][b];
        }
        if (P.owner()) {
            sm.m[t] = a.m[b];
            sm.R[t] = a.radius ? a.radius[b] : 0.0;
            sm.idx[t] = b;
            for (int l = 0; l < a.nlev; ++l)
                sm.irc[l][t] = rcp2(a.rc[l][b]);
            sm.rcd[t] = rcd;
        }
        {
            const double tr = wave_max_all(rcd);
            if (lane == 0 && P.owner()) sm.trho[t >> 6] = tr;
        }
        bool failed;
        [[clang::always_inline]] failed = bs_run(a, P, y);
        if (failed && threadIdx.x == 0) atomicOr(a.status, ST_NOCONV);
        if (P.owner()) {
            bs_store(a, b, y);
            if (a.radius) {
                a.m[b] = sm.m[t];
                a.radius[b] = sm.R[t];
            }
        }
        __syncthreads();   // LDS reuse by the next group
    }
}

// ---------------------------------------------------------------------------
// Groups of more than GROUP_BLOCK bodies (Sect. 6.1: the method that spreads
// one group over many thread blocks).  The paper drives each sub-step of
// that method from the host; here one persistent launch integrates the
// listed groups one after another, its workgroups meeting at a grid-wide
// barrier before every evaluation that reads other members' positions and
// at every group-wide maximum or minimum.  One thread per member (so a
// group may hold up to GENGA_GROUP_MAX bodies with the launch's workgroups
// all resident); the members are first ordered by a 64 x 64 cell grid over
// the group's x-y extent (cells along Hilbert's curve, members of a cell by their
// rank in the group), so that each wave's 64 members form a compact tile.
// A derivative then visits, per tile, only the tiles whose bounding boxes
// come within the larger deepest-level critical radius of the two tiles:
// every pair of the tiles left out has R = 0 exactly (the deepest level's
// factor 1 - K is zero at r >= rho), so its terms are exact zeros and the
// sums equal the all-pairs ones; a member's sum runs over its partners in
// ascending tile and slot order.
// ---------------------------------------------------------------------------
constexpr int GT = 256;             // threads per workgroup of the grid solver
constexpr int GCELL = 64;           // ordering cells per axis
// a barrier that has waited this long (wall clock, 100 MHz ticks: 2 s) gives up
constexpr uint64_t GWAIT_TICKS = 200000000ull;

struct GridDev {
    int32_t cap;                        // members per group the launch can hold
    const int32_t *big;                 // [0] listed groups, [1 ..] their roots
    double *pub;                        // [2][6][cap] published states (by parity)
    double *box;                        // [2][cap / 64][8] tile box lo, hi, max radius
    double *trho;                       // [cap / 64] largest deepest-level rc per tile
    double *mm, *mR;                    // [cap] member mass, radius
    double *mirc;                       // [GENGA_MAX_LEVELS][cap] 1 / rc per level
    double *mrc;                        // [cap] deepest-level rc
    int32_t *midx;                      // [cap] member body
    double *bpart;                      // [cap / 64][4] workgroup x-y extents
    int32_t *ccnt, *cfill;              // [GCELL^2] members per cell, fill counters
    int32_t *ctmp;                      // [cap] members by cell in arrival order
    unsigned long long *sync;           // [0] arrivals, [1] abort, [2..4] max slots
    long long *rmin;                    // [3] min slots
};

struct GridSmem {
    double sx[4][64], sy[4][64], sz[4][64], sm[4][64], src[4][64];
    double sirc[4][GENGA_MAX_LEVELS][64];
    double oirc[GENGA_MAX_LEVELS][GT];   // own 1 / rc per level
    double part[4][3][64];               // partial sums of the split waves
    double red[4][4];
    int32_t cstart[GCELL * GCELL];
    double ext[4];
    int64_t scan[GT / 64];
    int dead;
};

// The grid solver's LDS (only k_bs_grid reaches it).  Declared at namespace
// scope so that the out-of-line evaluation addresses it as LDS.
static __shared__ GridSmem g_gsm;

// Position of cell (x, y) of the GCELL x GCELL grid along Hilbert's curve
// (the usual construction: at each scale s the quadrant's number goes into
// the index, then the coordinates are turned into that quadrant's frame),
// so that consecutive cells along the order are always neighbours.
__device__ __forceinline__ unsigned hilbert_cell(unsigned x, unsigned y)
{
    unsigned d = 0;
    for (unsigned s = GCELL / 2; s > 0; s >>= 1) {
        const unsigned rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = GCELL - 1 - x;
                y = GCELL - 1 - y;
            }
            const unsigned tmp = x;
            x = y;
            y = tmp;
        }
    }
    return d;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct GridPol {
    const GridDev &G;
    int t, g, nlev, nblk;
    int split, sub;             // waves per tile, this wave's share (0: the owner)
    unsigned long long nbar;    // barriers passed in this launch
    int par;                    // parity of the last publication
    int nred;                   // reductions done in this launch
    bool dead;
    double m, R;                // own mass and radius
    double rcd;                 // own deepest-level rc

    __device__ bool member() const { return t < g; }
    // the first wave of a tile writes; the others hold copies of its members
    __device__ bool owner() const { return t < g && sub == 0; }
    __device__ int self() const { return t; }

    // Grid-wide barrier of the nblk workgroups: every arrival is counted
    // once after a release fence; the wait polls with relaxed loads (an
    // acquire per poll would invalidate the L2 of the poller's XCD each
    // time) and ends with one acquire fence.  The wait is bounded in wall
    // clock time: a barrier that times out (or finds that another workgroup
    // gave up) marks the launch dead, after which no barrier waits and the
    // flow fails to converge.
    __device__ bool sync()
    {
        __syncthreads();
        ++nbar;
        if (threadIdx.x == 0) {
            int d = dead ? 1 : 0;
            if (!d) {
                unsigned long long *cnt = G.sync;
                const unsigned long long target = nbar * (unsigned long long)nblk;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (__hip_atomic_load(cnt + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        d = 1;
                        break;
                    }
                    if (wall_clock64() - t0 > GWAIT_TICKS) {
                        __hip_atomic_store(cnt + 1, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        d = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            g_gsm.dead = d;
        }
        __syncthreads();
        dead = g_gsm.dead != 0;
        return !dead;
    }

    // the own tile's box (lo, hi) of positions z (members only)
    __device__ void tile_box(const double z[3], double lo[3], double hi[3]) const
    {
        const bool mem = member();
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = wave_min_all(mem ? z[c] : INFINITY);
            hi[c] = wave_max_all(mem ? z[c] : -INFINITY);
        }
    }

    __device__ void publish_n(const double z[6], int nc, double lo[3], double hi[3])
    {
        par ^= 1;
        double *P = G.pub + (size_t)par * 6 * G.cap;
        if (owner())
            for (int c = 0; c < nc; ++c) P[(size_t)c * G.cap + t] = z[c];
        tile_box(z, lo, hi);
        const double rmax = wave_max_all(member() ? R : 0.0);
        if ((threadIdx.x & 63) == 0 && owner()) {
            double *B = G.box + ((size_t)par * (G.cap / 64) + (t >> 6)) * 8;
            B[0] = lo[0]; B[1] = lo[1]; B[2] = lo[2];
            B[3] = hi[0]; B[4] = hi[1]; B[5] = hi[2];
            B[6] = rmax;
        }
        sync();
    }

    __device__ void publish(const double z[6])
    {
        double lo[3], hi[3];
        publish_n(z, 6, lo, hi);
    }

    __device__ void get(int q, double o[6]) const
    {
        const double *P = G.pub + (size_t)par * 6 * G.cap;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = P[(size_t)c * G.cap + q];
    }
    __device__ double mass(int q) const { return G.mm[q]; }
    __device__ double rad(int q) const { return G.mR[q]; }
    __device__ int idx(int q) const { return G.midx[q]; }
    __device__ void set_own(double mm, double RR)
    {
        if (member()) {
            m = mm;
            R = RR;
            if (owner()) {
                G.mm[t] = mm;
                G.mR[t] = RR;
            }
        }
    }


    // (one copy of the evaluation: bs_step reaches it from nine places; the
    // loop works on locals and LDS only).  A partner tile is visited if its
    // box comes within the larger deepest-level radius of the own tile's box
    // and of some member's own position (both tests skip only exact zeros).
    // The split waves of a tile take every split-th tile of its list each;
    // their partial sums are added in share order.
    __device__ __noinline__ void deriv(const BsDev &a, const double z[6], double f[6])
    {
        f[0] = z[3];
        f[1] = z[4];
        f[2] = z[5];
        double lo[3], hi[3];
        publish_n(z, 3, lo, hi);
        const double x0 = z[0], y0 = z[1], z0 = z[2];
        double ax = 0.0, ay = 0.0, az = 0.0;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int me = t, ng = g, nl = nlev, S_ = split, mine = sub;
        const int t0 = me - lane;
        GridSmem &S = g_gsm;
        if (!dead && t0 < ng) {
            const double Gc = a.G, rcme = rcd;
            const size_t cap = (size_t)G.cap;
            const int nt = (ng + 63) >> 6;
            const double *trho = G.trho, *mm = G.mm, *mrc = G.mrc, *mirc = G.mirc;
            const double rhoI = trho[t0 >> 6];
            const double *P = G.pub + (size_t)par * 6 * cap;
            const double *Bx = G.box + (size_t)par * (cap / 64) * 8;
            const double pos[3] = {x0, y0, z0};
            const bool mem = me < ng;
            int seen = 0;   // tiles of the list met so far (wave-uniform)
            for (int jb = 0; jb < nt; jb += 64) {
                const int Jl = jb + lane;
                bool near = false;
                double bj[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, rj = 0.0;
                if (Jl < nt) {
                    const double *B = Bx + (size_t)Jl * 8;
#pragma unroll
                    for (int c = 0; c < 6; ++c) bj[c] = B[c];
                    rj = trho[Jl];
                    const double rr = rhoI > rj ? rhoI : rj;
                    // (a NaN box keeps the tile: the flow then fails as a whole)
                    near = !(box_gap2(lo, hi, bj) > rr * rr * (1.0 + 0x1p-18));
                }
                unsigned long long mask = __ballot(near);
                while (mask) {
                    const int src = __builtin_ctzll(mask);
                    const int J = jb + src;
                    mask &= mask - 1;
                    // the same test for each member's own position: a tile whose
                    // box is large (members from distant cells) passes the box
                    // test against many tiles, of which few come near a member
                    double bJ[6];
#pragma unroll
                    for (int c = 0; c < 6; ++c) bJ[c] = __shfl(bj[c], src, 64);
                    const double rJ = __shfl(rj, src, 64);
                    const double rm = rcme > rJ ? rcme : rJ;
                    const bool close = mem && !(box_gap2(pos, pos, bJ) > rm * rm * (1.0 + 0x1p-18));
                    if (__ballot(close) == 0ull) continue;
                    if (seen++ % S_ != mine) continue;
                    const int jq = J * 64 + lane;
                    if (jq < ng) {
                        S.sx[w][lane] = P[jq];
                        S.sy[w][lane] = P[cap + jq];
                        S.sz[w][lane] = P[2 * cap + jq];
                        S.sm[w][lane] = mm[jq];
                        S.src[w][lane] = mrc[jq];
                        for (int l = 0; l < nl; ++l) S.sirc[w][l][lane] = mirc[(size_t)l * cap + jq];
                    }
                    wave_sync_lds();
                    const int qn = ng - J * 64 < 64 ? ng - J * 64 : 64;
                    const int qself = me - J * 64;
                    for (int q = 0; q < qn; ++q) {
                        if (q == qself) continue;
                        const double dx = S.sx[w][q] - x0, dy = S.sy[w][q] - y0,
                                     dz = S.sz[w][q] - z0;
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        const double rq = rcme > S.src[w][q] ? rcme : S.src[w][q];
                        // beyond the larger deepest-level radius R = 0 exactly
                        if (r2 > rq * rq * (1.0 + 0x1p-18)) continue;
                        const double ir = rsq2(r2);
                        const double Rw = bs_remainder(r2 * ir, &S.oirc[0][threadIdx.x], GT,
                                                       &S.sirc[w][0][q], 64, nl);
                        const double s = Gc * S.sm[w][q] * Rw * (ir * ir * ir);
                        ax += s * dx;
                        ay += s * dy;
                        az += s * dz;
                    }
                    wave_sync_lds();
                }
            }
        }
        // the star's pull, then the shares' partial sums in share order
        double kx = 0.0, ky = 0.0, kz = 0.0;
        if (member()) {
            const double r2s = x0 * x0 + y0 * y0 + z0 * z0;
            const double irs = rsq2(r2s);
            const double ks = -a.mu * (irs * irs * irs);
            kx = ks * x0;
            ky = ks * y0;
            kz = ks * z0;
        }
        if (S_ > 1) {
            S.part[w][0][lane] = ax;
            S.part[w][1][lane] = ay;
            S.part[w][2][lane] = az;
            __syncthreads();
            const int w0 = w - mine;
            for (int k = 0; k < S_; ++k) {
                kx += S.part[w0 + k][0][lane];
                ky += S.part[w0 + k][1][lane];
                kz += S.part[w0 + k][2][lane];
            }
            __syncthreads();
        } else {
            kx += ax;
            ky += ay;
            kz += az;
        }
        f[3] = kx;
        f[4] = ky;
        f[5] = kz;
    }

    // group-wide reductions through rotating slots: slot nred % 3 collects
    // this reduction; after its barrier workgroup 0 resets slot
    // (nred + 2) % 3, whose last readers have all passed this barrier and
    // whose next writers come after the next one (the split waves hold the
    // same values: a maximum or minimum counts them once)
    __device__ void reset_slot()
    {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const int s2 = (nred + 2) % 3;
            __hip_atomic_store(G.sync + 2 + s2, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(G.rmin + s2, NO_PAIR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ++nred;
    }

    __device__ double gmax(double v)
    {
        // non-negative (or +inf) values: their bit patterns order as integers
        v = wave_max_all(v);
        const int s = nred % 3;
        if ((threadIdx.x & 63) == 0 && !dead)
            __hip_atomic_fetch_max(G.sync + 2 + s, (unsigned long long)__double_as_longlong(v),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sync();
        double r = INFINITY;
        if (!dead)
            r = __longlong_as_double((long long)__hip_atomic_load(G.sync + 2 + s, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT));
        reset_slot();
        return r;
    }

    __device__ long long gmin(long long v)
    {
        for (int d = 32; d > 0; d >>= 1) {
            const long long o = __shfl_xor(v, d, 64);
            v = o < v ? o : v;
        }
        const int s = nred % 3;
        if ((threadIdx.x & 63) == 0 && !dead && v != NO_PAIR)
            __hip_atomic_fetch_min(G.rmin + s, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sync();
        long long r = NO_PAIR;
        if (!dead) r = __hip_atomic_load(G.rmin + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        reset_slot();
        return r;
    }

    __device__ long long overlap(const BsDev &a, const double z[6]);
};

// The grid solver's overlap search: tiles whose boxes stay apart by more
// than the sum of their largest radii hold no overlapping pair.
__device__ long long GridPol::overlap(const BsDev &a, const double z[6])
{
    double lo[3], hi[3];
    publish_n(z, 6, lo, hi);
    long long key = NO_PAIR;
    const int lane = threadIdx.x & 63;
    const int t0 = t - lane;
    if (!dead && t0 < g) {
        const int nt = (g + 63) >> 6;
        const double *Pp = G.pub + (size_t)par * 6 * G.cap;
        const double *Bx = G.box + (size_t)par * (G.cap / 64) * 8;
        const double rI = wave_max_all(member() ? R : 0.0);
        for (int jb = 0; jb < nt; jb += 64) {
            const int Jl = jb + lane;
            bool near = false;
            if (Jl < nt) {
                const double rs = rI + Bx[(size_t)Jl * 8 + 6];
                near = rs > 0.0 && !(box_gap2(lo, hi, Bx + (size_t)Jl * 8) > rs * rs * (1.0 + 0x1p-18));
            }
            unsigned long long mask = __ballot(near);
            while (mask) {
                const int J = jb + __builtin_ctzll(mask);
                mask &= mask - 1;
                const int qn = g - J * 64 < 64 ? g - J * 64 : 64;
                for (int qq = 0; qq < qn; ++qq) {
                    const int q = J * 64 + qq;
                    if (!member() || q <= t || key != NO_PAIR) continue;
                    const double rs = R + G.mR[q];
                    const double dx = Pp[q] - z[0], dy = Pp[(size_t)G.cap + q] - z[1],
                                 dz = Pp[2 * (size_t)G.cap + q] - z[2];
                    if (rs > 0.0 && dx * dx + dy * dy + dz * dz < rs * rs)
                        key = (long long)t * KEY_BASE + q;
                }
            }
        }
    }
    return gmin(key);
}

// Spatial order of the group's members (see above): by cell, then by body
// index, whatever the order of the group's slots; perm[k] = body of the k-th
// member in that order.  Four grid barriers; only the owners contribute.
__device__ void grid_order(const BsDev &a, GridPol &P, int32_t root, int32_t *perm)
{
    const GridDev &G = P.G;
    GridSmem &S = g_gsm;
    const int t = P.t;
    const bool own = P.owner();
    const int nthr = P.nblk * GT;
    const int tid = blockIdx.x * GT + threadIdx.x;
    const int32_t b = own ? a.gmem[a.gstart[root] + t] : 0;
    double x = 0.0, y = 0.0;
    if (own) {
        x = a.shadow[b];
        y = a.shadow[(size_t)a.n + b];
    }
    for (int c = tid; c < GCELL * GCELL; c += nthr) {
        G.ccnt[c] = 0;
        G.cfill[c] = 0;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    {
        const double v[4] = {wave_min_all(own ? x : INFINITY), wave_max_all(own ? x : -INFINITY),
                             wave_min_all(own ? y : INFINITY), wave_max_all(own ? y : -INFINITY)};
        if (lane == 0)
            for (int c = 0; c < 4; ++c) S.red[w][c] = v[c];
        __syncthreads();
        if (threadIdx.x < 4) {
            const int c = threadIdx.x;
            double r = S.red[0][c];
            for (int k = 1; k < 4; ++k) r = (c & 1) ? (S.red[k][c] > r ? S.red[k][c] : r)
                                                    : (S.red[k][c] < r ? S.red[k][c] : r);
            G.bpart[(size_t)blockIdx.x * 4 + c] = r;
        }
    }
    P.sync();
    // the group's extent (the same arithmetic in every workgroup)
    double *ext = S.ext;
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        double r = G.bpart[c];
        for (int k = 1; k < P.nblk; ++k) {
            const double o = G.bpart[(size_t)k * 4 + c];
            r = (c & 1) ? (o > r ? o : r) : (o < r ? o : r);
        }
        ext[c] = r;
    }
    __syncthreads();
    unsigned cell = 0;
    if (own) {
        const double wx = ext[1] - ext[0], wy = ext[3] - ext[2];
        const double fx = wx > 0.0 ? (x - ext[0]) * (GCELL / wx) : 0.0;
        const double fy = wy > 0.0 ? (y - ext[2]) * (GCELL / wy) : 0.0;
        int cx = fx >= 0.0 ? (int)fx : 0, cy = fy >= 0.0 ? (int)fy : 0;
        cx = cx < GCELL - 1 ? cx : GCELL - 1;
        cy = cy < GCELL - 1 ? cy : GCELL - 1;
        // (NaN positions land in cell 0: the flow fails later anyway)
        cell = hilbert_cell((unsigned)cx, (unsigned)cy);
        atomicAdd(G.ccnt + cell, 1);
    }
    P.sync();
    // exclusive scan of the cell counts, in every workgroup
    {
        constexpr int PER = GCELL * GCELL / GT;
        int loc[PER], sum = 0;
        for (int k = 0; k < PER; ++k) {
            loc[k] = __hip_atomic_load(G.ccnt + threadIdx.x * PER + k, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            sum += loc[k];
        }
        int64_t tot;
        int64_t off = block_excl_scan<GT>((int64_t)sum, &tot, S.scan);
        for (int k = 0; k < PER; ++k) {
            S.cstart[threadIdx.x * PER + k] = (int32_t)off;
            off += loc[k];
        }
    }
    __syncthreads();
    if (own) G.ctmp[S.cstart[cell] + atomicAdd(G.cfill + cell, 1)] = b;
    P.sync();
    // within a cell by body index (the slots' arrival order is not fixed)
    if (own) {
        const int c0 = S.cstart[cell];
        const int cn = __hip_atomic_load(G.ccnt + cell, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int rank = 0;
        for (int k = c0; k < c0 + cn; ++k) rank += G.ctmp[k] < b;
        perm[c0 + rank] = b;
    }
    P.sync();
}

// Waves per tile for a group of g members when nb workgroups (of 4 waves)
// can take part: the most of 4, 2, 1 that fit in them (0: the group does not
// fit).
__device__ inline int grid_split(int g, int nb)
{
    const int nt = (g + 63) / 64;
    for (int s = 4; s >= 1; s >>= 1)
        if ((nt * s + 3) / 4 <= nb) return s;
    return 0;
}

// All listed groups of more than GROUP_BLOCK bodies, one after another.
// Launched with as many workgroups as are resident together (sized for two
// per compute unit); a group takes the most waves per tile that fit, and the
// workgroups beyond the largest group's need return at once.
__global__ __launch_bounds__(GT, 2) void k_bs_grid(BsDev a, GridDev G)
{
    GridSmem &S = g_gsm;
    const int nbig = G.big[0];
    int need = 0;
    for (int k = 0; k < nbig; ++k) {
        const int g = a.gsize[G.big[1 + k]];
        const int s = g <= G.cap ? grid_split(g, gridDim.x) : 0;
        if (s) {
            const int nb = ((g + 63) / 64 * s + 3) / 4;
            need = nb > need ? nb : need;
        } else if (blockIdx.x == 0 && threadIdx.x == 0) {
            atomicOr(a.status, ST_GROUP);
        }
    }
    if ((int)blockIdx.x >= need) return;
    GridPol P{G};
    P.nlev = a.nlev;
    P.nblk = need;
    P.nbar = 0;
    P.par = 0;
    P.nred = 0;
    P.dead = false;
    int32_t *perm = G.ctmp + G.cap;   // second half of the cell scratch
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int k = 0; k < nbig; ++k) {
        const int32_t root = G.big[1 + k];
        const int g = a.gsize[root];
        const int split = g <= G.cap ? grid_split(g, gridDim.x) : 0;
        if (!split) continue;
        P.g = g;
        P.split = split;
        P.sub = gw % split;
        P.t = gw / split * 64 + lane;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            atomicAdd(a.gstats, 1ull);
            atomicMax(a.gstats + 1, (unsigned long long)g);
        }
        grid_order(a, P, root, perm);
        const int t = P.t;
        const bool mem = t < g;
        const int32_t b = mem ? perm[t] : 0;
        double y[6] = {0, 0, 0, 0, 0, 0};
        P.m = 0.0;
        P.R = 0.0;
        P.rcd = 0.0;
        if (mem) {
#pragma unroll
            for (int c = 0; c < 6; ++c) y[c] = a.shadow[(size_t)c * a.n + b];
            P.m = a.m[b];
            P.R = a.radius ? a.radius[b] : 0.0;
            P.rcd = a.rc[a.nlev - 1][b];
            for (int l = 0; l < a.nlev; ++l) {
                const double ir = rcp2(a.rc[l][b]);
                S.oirc[l][threadIdx.x] = ir;
                if (P.owner()) G.mirc[(size_t)l * G.cap + t] = ir;
            }
            if (P.owner()) {
                G.mm[t] = P.m;
                G.mR[t] = P.R;
                G.mrc[t] = P.rcd;
                G.midx[t] = b;
            }
        }
        const double tr = wave_max_all(mem ? P.rcd : 0.0);
        if (lane == 0 && P.owner()) G.trho[t >> 6] = tr;
        // (the first evaluation's barrier publishes these)
        const bool failed = bs_run(a, P, y);
        if (failed && t == 0) atomicOr(a.status, ST_NOCONV);
        if (P.owner()) {
            bs_store(a, b, y);
            if (a.radius) {
                a.m[b] = P.m;
                a.radius[b] = P.R;
            }
        }
        P.sync();   // scratch reuse by the next group
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

// Groups of list l and their members' state saved into shadow[l].
static hipError_t group_and_save(const LevelRun &R, int l)
{
    const LevelLayout &V = *R.V;
    const int64_t n = R.b->n;
    const unsigned nt = (unsigned)((n + LT - 1) / LT);
    int32_t *lab = R.at<int32_t>(V.glab), *flag = R.at<int32_t>(V.gflag);
    int32_t *gsize = R.at<int32_t>(V.gsize), *gfill = R.at<int32_t>(V.gfill);
    int32_t *gstart = R.at<int32_t>(V.gstart), *groot = R.at<int32_t>(V.groot);
    int32_t *gtmp = R.at<int32_t>(V.gtmp), *gmem = R.at<int32_t>(V.gmem);
    int32_t *gcount = R.at<int32_t>(V.gcount);
    int64_t *tsum = R.at<int64_t>(V.gtsum);
    const int32_t *pi = R.at<int32_t>(V.pi[l]), *pj = R.at<int32_t>(V.pj[l]);
    const int64_t *cnt = R.at<int64_t>(V.cnt) + l;
    // the union-find's parents live in gtmp until the roots are known
    hipLaunchKernelGGL(k_group_init, dim3(LG), dim3(LT), 0, R.s, gtmp, flag, gsize, gfill, n);
    hipLaunchKernelGGL(k_group_union, dim3(LG), dim3(LT), 0, R.s, pi, pj, cnt, V.cap, gtmp, flag);
    hipLaunchKernelGGL(k_group_root, dim3(LG), dim3(LT), 0, R.s, gtmp, flag, lab, gsize, n);
    hipLaunchKernelGGL(k_group_tiles, dim3(nt), dim3(LT), 0, R.s, flag, lab, gsize, n, tsum);
    int32_t *big = V.gbig ? R.at<int32_t>(V.gbig) : nullptr;
    unsigned long long *gsync = V.gbig ? R.at<unsigned long long>(V.gsync) : nullptr;
    hipLaunchKernelGGL(k_group_top, dim3(1), dim3(ST), 0, R.s, tsum, (int64_t)nt, gcount, big, gsync);
    hipLaunchKernelGGL(k_group_write, dim3(nt), dim3(LT), 0, R.s, flag, lab, gsize, n, tsum, gstart,
                       groot, big);
    hipLaunchKernelGGL(k_group_fill, dim3(LG), dim3(LT), 0, R.s, flag, lab, gstart, gfill, gtmp, n);
    hipLaunchKernelGGL(k_group_rank, dim3(LG), dim3(LT), 0, R.s, lab, gstart, gsize, gtmp, gcount,
                       gmem);
    BodyDev mem = R.bodies_of(0);
    mem.bodies = gmem;
    mem.nbod = gcount + 1;
    hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, R.s, mem, R.at<double>(V.shadow[l]), n,
                       1);
    return hipGetLastError();
}

// Workgroups of k_bs_grid that the current device holds at once (queried
// once per device).
static hipError_t grid_resident_blocks(int *out)
{
    static std::mutex mu;
    static int cached[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (!cached[dev]) {
        int per_cu = 0, cus = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bs_grid, GT, 0)) !=
            hipSuccess)
            return e;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
            hipSuccess)
            return e;
        if (per_cu < 1 || cus < 1) return hipErrorLaunchFailure;
        cached[dev] = per_cu * cus;
    }
    *out = cached[dev];
    return hipSuccess;
}

// The groups of list l over dt_l from the saved state, weights of levels 0..l.
static hipError_t direct_solve(const LevelRun &R, int l, double dt_l)
{
    const LevelLayout &V = *R.V;
    BsDev a;
    a.groot = R.at<int32_t>(V.groot);
    a.gstart = R.at<int32_t>(V.gstart);
    a.gsize = R.at<int32_t>(V.gsize);
    a.gmem = R.at<int32_t>(V.gmem);
    a.gcount = R.at<int32_t>(V.gcount);
    a.shadow = R.at<double>(V.shadow[l]);
    a.n = R.b->n;
    a.x = R.b->x; a.y = R.b->y; a.z = R.b->z;
    a.vx = R.b->vx; a.vy = R.b->vy; a.vz = R.b->vz;
    a.m = R.b->m;
    for (int q = 0; q < GENGA_MAX_LEVELS; ++q) a.rc[q] = nullptr;
    a.rc[0] = R.b->rc;
    for (int q = 1; q <= l; ++q) a.rc[q] = R.at<double>(V.rc[q]);
    a.nlev = l + 1;
    a.G = R.p->G;
    a.mu = R.p->G * R.p->m_star;
    a.H = dt_l;
    a.eps = R.p->bs_eps > 0.0 ? R.p->bs_eps : 1e-12;
    a.status = R.status();
    a.gstats = R.at<unsigned long long>(V.gstats);
    a.radius = R.b->R;
    a.coll_tol = R.p->coll_tol > 0.0 ? R.p->coll_tol : 1e-6;
    a.coll_i = R.at<int32_t>(V.coll_i);
    a.coll_j = R.at<int32_t>(V.coll_j);
    a.coll_du = R.at<double>(V.coll_du);
    a.coll_count = R.at<unsigned long long>(V.coll_count);
    a.coll_cap = LEVEL_COLL_CAP;
    hipLaunchKernelGGL(k_bs_lanes<BS_GS>, dim3(LG), dim3(LT), 0, R.s, a);
    // groups of more than 8 bodies are rare at the deepest level: one
    // launch of 512-thread workgroups takes all of them (an empty launch per
    // class cost ~4.5 us per deepest sub-step)
    hipLaunchKernelGGL(k_bs<GROUP_BLOCK>, dim3(LG_BIG), dim3(GROUP_BLOCK), 0, R.s, a, BS_GS);
    if (!V.gbig) return hipGetLastError();
    // groups beyond one workgroup: as many workgroups as fit the capacity
    // and are resident on the device together (the barriers need them all)
    int resident = 0;
    hipError_t e = grid_resident_blocks(&resident);
    if (e != hipSuccess) return e;
    const int nb = (int)std::min<int64_t>(V.gcap / 64, resident);
    GridDev G;
    G.cap = (int32_t)std::min<int64_t>(V.gcap, (int64_t)nb * GT);
    G.big = R.at<int32_t>(V.gbig);
    G.pub = R.at<double>(V.gpub);
    G.box = R.at<double>(V.gbox);
    G.trho = R.at<double>(V.gtrho);
    G.mm = R.at<double>(V.gmm);
    G.mR = R.at<double>(V.gmR);
    G.mrc = R.at<double>(V.gmrc);
    G.mirc = R.at<double>(V.gmirc);
    G.midx = R.at<int32_t>(V.gmidx);
    G.bpart = R.at<double>(V.gbpart);
    G.ccnt = R.at<int32_t>(V.gccnt);
    G.cfill = R.at<int32_t>(V.gcfill);
    G.ctmp = R.at<int32_t>(V.gctmp);
    G.sync = R.at<unsigned long long>(V.gsync);
    G.rmin = (long long *)(G.sync + 5);
    hipLaunchKernelGGL(k_bs_grid, dim3(nb), dim3(GT), 0, R.s, a, G);
    return hipGetLastError();
}

// Level l >= 1 over list l - 1, sub-steps of dt_l.
static hipError_t advance(const LevelRun &R, int l, double dt_l)
{
    const LevelLayout &V = *R.V;
    const genga_params *p = R.p;
    const int64_t n = R.b->n;
    const bool deeper = l < V.L - 1;
    const bool direct = V.direct && l == V.L - 1;
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
        if (direct && (e = group_and_save(R, l)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_drift_list, dim3(LG), dim3(LT), 0, R.s, up, p->G * p->m_star, dt_l);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (deeper) {
            hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, R.s, R.bodies_of(l),
                               R.at<double>(V.shadow[l]), n, 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = advance(R, l + 1, dt_l / p->substeps)) != hipSuccess) return e;
        }
        if (direct && (e = direct_solve(R, l, dt_l)) != hipSuccess) return e;
        if ((e = level_kick(R, l, 0.5 * dt_l)) != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

LevelLayout make_level_layout(int64_t n, const genga_params *p, size_t base)
{
    LevelLayout V;
    if (!p || (p->slevels < 2 && !p->direct)) {
        V.total = base;
        return V;
    }
    V.L = p->slevels > 1 ? p->slevels : 1;
    V.direct = p->direct ? 1 : 0;
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
    if (V.direct) {
        V.shadow[V.L - 1] = take(sizeof(double) * 6 * (size_t)n);
        V.glab = take(sizeof(int32_t) * (size_t)n);
        V.gflag = take(sizeof(int32_t) * (size_t)n);
        V.gsize = take(sizeof(int32_t) * (size_t)n);
        V.gfill = take(sizeof(int32_t) * (size_t)n);
        V.gstart = take(sizeof(int32_t) * (size_t)n);
        V.groot = take(sizeof(int32_t) * (size_t)n);
        V.gtmp = take(sizeof(int32_t) * (size_t)n);
        V.gmem = take(sizeof(int32_t) * (size_t)n);
        V.gcount = take(sizeof(int32_t) * 2);
        V.gstats = take(sizeof(int64_t) * 2);
        V.coll_count = take(sizeof(int64_t));
        V.coll_i = take(sizeof(int32_t) * LEVEL_COLL_CAP);
        V.coll_j = take(sizeof(int32_t) * LEVEL_COLL_CAP);
        V.coll_du = take(sizeof(double) * LEVEL_COLL_CAP);
        V.gtsum = take(sizeof(int64_t) * 2 * (size_t)((n + LT - 1) / LT));
        if (n > GROUP_BLOCK) {
            const int64_t gc = (n + GT - 1) / GT * GT;
            V.gcap = gc < GENGA_GROUP_MAX ? gc : GENGA_GROUP_MAX;
            const size_t c = (size_t)V.gcap;
            V.gbig = take(sizeof(int32_t) * (size_t)(2 + n / (GROUP_BLOCK + 1)));
            V.gsync = take(sizeof(uint64_t) * 8);
            V.gpub = take(sizeof(double) * 12 * c);
            V.gbox = take(sizeof(double) * 2 * (c / 64) * 8);
            V.gtrho = take(sizeof(double) * (c / 64));
            V.gmm = take(sizeof(double) * c);
            V.gmR = take(sizeof(double) * c);
            V.gmrc = take(sizeof(double) * c);
            V.gmirc = take(sizeof(double) * (size_t)V.L * c);
            V.gmidx = take(sizeof(int32_t) * c);
            V.gbpart = take(sizeof(double) * 4 * (c / 64));
            V.gccnt = take(sizeof(int32_t) * GCELL * GCELL);
            V.gcfill = take(sizeof(int32_t) * GCELL * GCELL);
            V.gctmp = take(sizeof(int32_t) * 2 * c);
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
    hipLaunchKernelGGL(k_level_begin, dim3(1), dim3(64), 0, s, R.at<int64_t>(V.lcount), V.L, cnt0,
                       V.direct ? R.at<int64_t>(V.gstats) : nullptr,
                       V.direct ? R.at<int64_t>(V.coll_count) : nullptr);
    if (out) {
        hipLaunchKernelGGL(k_copy_pairs, dim3(LG), dim3(LT), 0, s, R.at<int32_t>(V.pi[0]),
                           R.at<int32_t>(V.pj[0]), cnt0, V.cap, out->i, out->j, out->capacity,
                           out->count, R.status());
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (V.L == 1) return group_and_save(R, 0);   // direct solver on E_0
    if ((e = build_adj(R, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, s, R.bodies_of(0),
                       R.at<double>(V.shadow[0]), b->n, 1);
    return hipGetLastError();
}

hipError_t levels_after_drift(genga_bodies *b, const genga_params *p, const LevelLayout &V,
                              char *ws, hipStream_t s)
{
    LevelRun R{b, p, &V, ws, s};
    if (V.L == 1) return direct_solve(R, 0, p->dt);
    hipLaunchKernelGGL(k_state_list, dim3(LG), dim3(LT), 0, s, R.bodies_of(0),
                       R.at<double>(V.shadow[0]), b->n, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return advance(R, 1, p->dt / p->substeps);
}

}  // namespace genga
