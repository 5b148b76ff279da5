// C ABI entry points of libgenga.so (declared in include/genga.h): argument
// checking, workspace layout and kernel sequencing on the caller's stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "genga_internal.h"

namespace genga {

static thread_local int g_last_hip = 0;

void set_hip_error(hipError_t e) { g_last_hip = (int)e; }

static int hip_fail(hipError_t e)
{
    set_hip_error(e);
    return GENGA_E_HIP;
}

static bool is_fin(double v) { return isfinite(v); }

static int check_bodies(const genga_bodies *b, bool need_v, bool need_rc)
{
    if (!b || b->n < 1 || b->n > (int64_t)INT32_MAX) return GENGA_E_INVAL;
    if (!b->x || !b->y || !b->z || !b->m) return GENGA_E_INVAL;
    if (need_v && (!b->vx || !b->vy || !b->vz)) return GENGA_E_INVAL;
    if (need_rc && !b->rc) return GENGA_E_INVAL;
    return GENGA_OK;
}

static int check_params(const genga_params *p)
{
    if (!p) return GENGA_E_INVAL;
    if (!is_fin(p->G) || p->G < 0.0) return GENGA_E_INVAL;
    if (!is_fin(p->m_star) || !(p->m_star > 0.0)) return GENGA_E_INVAL;
    if (!is_fin(p->dt) || !is_fin(p->n1) || !is_fin(p->n2)) return GENGA_E_INVAL;
    if (p->n1 < 0.0 || p->n2 < 0.0) return GENGA_E_INVAL;
    if (p->precision != GENGA_FP64 && p->precision != GENGA_MIXED) return GENGA_E_INVAL;
    if (p->ipt < 0 || p->ipt > 2 || p->slices < 0) return GENGA_E_INVAL;
    if ((p->flags & GENGA_FLAG_DIRECTED) && (p->flags & GENGA_FLAG_SYMMETRIC)) return GENGA_E_INVAL;
    if (p->block < 0 || p->tile_cols < 0 || p->grid < 0) return GENGA_E_INVAL;
    if (p->tp_mode < 0 || p->tp_mode > 2 || p->n_massive < 0) return GENGA_E_INVAL;
    if (p->slevels < 0 || p->slevels > GENGA_MAX_LEVELS) return GENGA_E_INVAL;
    if (!is_fin(p->c_light) || p->c_light < 0.0) return GENGA_E_INVAL;
    if (!is_fin(p->coll_tol) || p->coll_tol < 0.0 || p->coll_tol >= 1.0) return GENGA_E_INVAL;
    if (p->direct != 0 && p->direct != 1) return GENGA_E_INVAL;
    if (!is_fin(p->bs_eps) || p->bs_eps < 0.0) return GENGA_E_INVAL;
    if (p->slevels > 1 || p->direct) {
        // adjacency offsets are int32 over 2 level_capacity entries
        if (p->level_capacity < 1 || p->level_capacity > (1 << 30)) return GENGA_E_INVAL;
        if (p->slevels > 1 && p->substeps < 1) return GENGA_E_INVAL;
    }
    return GENGA_OK;
}

// Test-particle modes: n_massive <= n; only the binary64 single-system kick,
// pair list and step support them.
static int check_tp(const genga_bodies *b, const genga_params *p, bool supported)
{
    if (p->tp_mode == 0) return GENGA_OK;
    if (p->n_massive > b->n) return GENGA_E_INVAL;
    if (!supported || p->precision != GENGA_FP64) return GENGA_E_UNSUPPORTED;
    return GENGA_OK;
}

// Bodies whose momentum enters HC: in test-particle mode 1 the test particles
// act on no body, so only the massive ones.
static int64_t hc_count(const genga_bodies *b, const genga_params *p)
{
    return p->tp_mode == 1 ? p->n_massive : b->n;
}

static int check_pairs(const genga_pairs *q)
{
    if (!q) return GENGA_OK;
    if (!q->count || q->capacity < 0) return GENGA_E_INVAL;
    if (q->capacity > 0 && (!q->i || !q->j)) return GENGA_E_INVAL;
    return GENGA_OK;
}

static int status_to_code(int32_t st)
{
    if (st & ST_RCRIT) return GENGA_E_RCRIT;
    if (st & ST_NONFINITE) return GENGA_E_NONFINITE;
    if (st & ST_NOCONV) return GENGA_E_NOCONV;
    if (st & ST_GROUP) return GENGA_E_GROUP;
    if (st & ST_OVERFLOW) return GENGA_E_OVERFLOW;
    return GENGA_OK;
}

// fuse_hc: also apply the Sun kick x += h P / m_star after the velocities,
// with P from the momentum partials in L.hc2 (genga_step's second half).
static int do_kick(const genga_bodies *b, const genga_params *p, double h, double *ax, double *ay,
                   double *az, genga_pairs *pairs, bool forces, void *ws, void *stream,
                   int ev_slot = 0, bool fuse_hc = false)
{
    const KickCfg c = choose_kick_cfg(b->n, p);
    const Layout L = make_layout(b->n, c);
    KickLaunch k;
    k.x = b->x; k.y = b->y; k.z = b->z; k.m = b->m; k.rc = b->rc;
    k.vx = b->vx; k.vy = b->vy; k.vz = b->vz;
    k.ax = ax; k.ay = ay; k.az = az;
    k.n = b->n;
    k.G = p->G;
    k.h = h;
    k.precision = p->precision;
    k.forces = forces;
    k.pairs = pairs;
    k.ev0 = p->prof_events[ev_slot];
    k.ev1 = p->prof_events[ev_slot + 1];
    k.hfac = 0.0;
    k.tiles = nullptr;
    k.sysid = nullptr;
    k.sys_slices = nullptr;
    k.sys_dt = nullptr;
    k.sys_off = nullptr;
    if (fuse_hc) {
        k.px = b->x; k.py = b->y; k.pz = b->z;
        k.hc_part = (const double *)((char *)ws + L.hc2);
        k.hc_nb = L.nb;
        k.hc_h = h;
        k.hc_m_star = p->m_star;
    }
    hipError_t e = launch_kick(k, c, L, (char *)ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return GENGA_OK;
}

// Scratch of genga_kick_static: one array per GPU, which holds it from the
// load of this library's code object until the process ends.  In host code
// its name is a host-side stand-in, never a device address: the device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[GENGA_STATIC_SCRATCH_BYTES];

constexpr int STATIC_MAX_DEVICES = 64;
static std::mutex g_static_mu;
static void *g_static_ptr[STATIC_MAX_DEVICES];

// Device address of this device's scratch array (the current device).
static int static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return GENGA_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!ptr) return GENGA_E_HIP;
        g_static_ptr[dev] = ptr;
    }
    *out = g_static_ptr[dev];
    return GENGA_OK;
}

// Status words at the head of the scratch (status, tile counter, refined
// rows, padding): cleared at the start of every call.
__global__ void k_static_begin(int32_t *head)
{
    if (threadIdx.x < 64) head[threadIdx.x] = 0;
}

// The call's status bits as the most severe return code, into *out.
__global__ void k_static_end(const int32_t *head, int32_t *out)
{
    const int32_t st = head[0];
    int32_t code = GENGA_OK;
    if (st & ST_RCRIT) code = GENGA_E_RCRIT;
    else if (st & ST_NONFINITE) code = GENGA_E_NONFINITE;
    else if (st & ST_NOCONV) code = GENGA_E_NOCONV;
    else if (st & ST_GROUP) code = GENGA_E_GROUP;
    else if (st & ST_OVERFLOW) code = GENGA_E_OVERFLOW;
    *out = code;
}

}  // namespace genga

using namespace genga;

extern "C" {

int genga_version(void) { return 100; }

const char *genga_strerror(int code)
{
    switch (code) {
    case GENGA_OK: return "ok";
    case GENGA_E_INVAL: return "invalid argument";
    case GENGA_E_OVERFLOW: return "encounter list longer than its capacity";
    case GENGA_E_NONFINITE: return "coincident bodies or non-finite result";
    case GENGA_E_HIP: return "HIP runtime error";
    case GENGA_E_UNSUPPORTED: return "unsupported option";
    case GENGA_E_NOCONV: return "Kepler solver or Bulirsch-Stoer did not converge";
    case GENGA_E_RCRIT: return "negative or non-finite critical radius";
    case GENGA_E_GROUP: return "close-encounter group larger than the direct solver's limit";
    case GENGA_E_SCRATCH:
        return "genga_kick_static: the kick needs more scratch than GENGA_STATIC_SCRATCH_BYTES";
    default: return "unknown error";
    }
}

int genga_last_hip_error(void) { return g_last_hip; }

size_t genga_workspace_bytes(int64_t n, const genga_params *p)
{
    if (n < 1) return 0;
    const KickCfg c = choose_kick_cfg(n, p);
    return make_level_layout(n, p, make_layout(n, c).total).total;
}

int genga_read_status(void *ws, void *stream)
{
    if (!ws) return GENGA_E_INVAL;
    int32_t st = 0;
    hipError_t e = hipMemcpyAsync(&st, ws, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    if (st) {
        e = launch_clear_status((char *)ws, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e);
    }
    return status_to_code(st);
}

int genga_clear_status(void *ws, void *stream)
{
    if (!ws) return GENGA_E_INVAL;
    hipError_t e = launch_clear_status((char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_rcrit(const genga_bodies *b, const genga_params *p, void *ws, void *stream)
{
    int r = check_bodies(b, true, true);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (!ws) return GENGA_E_INVAL;
    hipError_t e = launch_rcrit(b, p, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_kick(const genga_bodies *b, const genga_params *p, double h, double *ax, double *ay,
               double *az, genga_pairs *pairs, void *ws, void *stream)
{
    int r = check_bodies(b, h != 0.0, true);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if ((r = check_pairs(pairs))) return r;
    if (!ws || !is_fin(h)) return GENGA_E_INVAL;
    if ((ax || ay || az) && !(ax && ay && az)) return GENGA_E_INVAL;
    if ((r = check_tp(b, p, true))) return r;
    return do_kick(b, p, h, ax, ay, az, pairs, true, ws, stream);
}

int genga_encounter_pairs(const genga_bodies *b, const genga_params *p, genga_pairs *pairs,
                          void *ws, void *stream)
{
    int r = check_bodies(b, false, true);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (!pairs) return GENGA_E_INVAL;
    if ((r = check_pairs(pairs))) return r;
    if (!ws) return GENGA_E_INVAL;
    if (p->tp_mode != 0 && p->n_massive > b->n) return GENGA_E_INVAL;
    return do_kick(b, p, 0.0, nullptr, nullptr, nullptr, pairs, false, ws, stream);
}

int genga_hc(genga_bodies *b, const genga_params *p, double h, void *ws, void *stream)
{
    int r = check_bodies(b, true, false);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (!ws || !is_fin(h)) return GENGA_E_INVAL;
    if (p->tp_mode != 0 && p->n_massive > b->n) return GENGA_E_INVAL;
    const Layout L = make_layout(b->n, choose_kick_cfg(b->n, p));
    hipError_t e = launch_hc(b, p->m_star, h, L, (char *)ws, (hipStream_t)stream, hc_count(b, p));
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_drift(genga_bodies *b, const genga_params *p, double dt, void *ws, void *stream)
{
    int r = check_bodies(b, true, false);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (!ws || !is_fin(dt)) return GENGA_E_INVAL;
    hipError_t e = launch_drift(b, p->G * p->m_star, dt, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_energy(const genga_bodies *b, const genga_params *p, double *out, void *ws,
                 void *stream)
{
    int r = check_bodies(b, true, false);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    if (!ws || !out) return GENGA_E_INVAL;
    const KickCfg c = choose_kick_cfg(b->n, p);
    const Layout L = make_layout(b->n, c);
    hipError_t e = launch_energy(b, p, out, c, L, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_energy_k(const genga_bodies *b, const genga_params *p, genga_pairs *pairs, double *out,
                   void *ws, void *stream)
{
    int r = check_bodies(b, true, true);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    if (!ws || !out || !pairs) return GENGA_E_INVAL;
    if ((r = check_pairs(pairs))) return r;
    const KickCfg c = choose_kick_cfg(b->n, p);
    const Layout L = make_layout(b->n, c);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_energy(b, p, out, c, L, (char *)ws, s);
    if (e != hipSuccess) return hip_fail(e);
    if ((r = do_kick(b, p, 0.0, nullptr, nullptr, nullptr, pairs, false, ws, stream))) return r;
    e = launch_energy_k_pairs(b, p, pairs, out, L, (char *)ws, s);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

static int check_adj(const genga_adjoint *adj, bool pos, bool vel, bool m, bool rc)
{
    if (!adj) return GENGA_E_INVAL;
    if (pos && (!adj->x || !adj->y || !adj->z)) return GENGA_E_INVAL;
    if (vel && (!adj->vx || !adj->vy || !adj->vz)) return GENGA_E_INVAL;
    if (m && !adj->m) return GENGA_E_INVAL;
    if (rc && !adj->rc) return GENGA_E_INVAL;
    return GENGA_OK;
}

int genga_kick_vjp(const genga_bodies *b, const genga_params *p, double scale, const double *abx,
                   const double *aby, const double *abz, genga_adjoint *adj, void *ws, void *stream)
{
    int r = check_bodies(b, false, true);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    if ((r = check_adj(adj, true, false, true, true))) return r;
    if (!ws || !abx || !aby || !abz || !is_fin(scale)) return GENGA_E_INVAL;
    hipError_t e = launch_kick_vjp(b, p, scale, abx, aby, abz, adj, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_rcrit_vjp(const genga_bodies *b, const genga_params *p, genga_adjoint *adj, void *ws,
                    void *stream)
{
    int r = check_bodies(b, true, false);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    if ((r = check_adj(adj, true, true, true, true))) return r;
    if (!ws) return GENGA_E_INVAL;
    hipError_t e = launch_rcrit_vjp(b, p, adj, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_hc_vjp(const genga_bodies *b, const genga_params *p, double h, genga_adjoint *adj,
                 void *ws, void *stream)
{
    int r = check_bodies(b, true, false);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    if ((r = check_adj(adj, true, true, true, false))) return r;
    if (!ws || !is_fin(h)) return GENGA_E_INVAL;
    const Layout L = make_layout(b->n, choose_kick_cfg(b->n, p));
    hipError_t e = launch_hc_vjp(b, p, h, adj, L, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_drift_vjp(const genga_bodies *b, const genga_params *p, double dt, genga_adjoint *adj,
                    void *ws, void *stream)
{
    int r = check_bodies(b, true, false);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    if ((r = check_adj(adj, true, true, false, false))) return r;
    if (!ws || !is_fin(dt)) return GENGA_E_INVAL;
    hipError_t e = launch_drift_vjp(b, p, dt, adj, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_step(genga_bodies *b, const genga_params *p, genga_pairs *pairs, void *ws, void *stream)
{
    int r = check_bodies(b, true, true);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if ((r = check_pairs(pairs))) return r;
    if (!ws) return GENGA_E_INVAL;
    if ((r = check_tp(b, p, true))) return r;
    const bool levels = p->slevels > 1 || p->direct;
    const bool gr = p->c_light > 0.0;
    if (levels && p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    if (gr && (levels || p->tp_mode != 0)) return GENGA_E_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const double h = 0.5 * p->dt;
    const Layout L = make_layout(b->n, choose_kick_cfg(b->n, p));
    const LevelLayout V = make_level_layout(b->n, p, L.total);
    genga_pairs e0;
    if (levels) e0 = level0_pairs(V, (char *)ws);
    hipError_t e = launch_rcrit(b, p, (char *)ws, s);
    if (e != hipSuccess) return hip_fail(e);
    if ((r = do_kick(b, p, h, nullptr, nullptr, nullptr, levels ? &e0 : pairs, true, ws, stream)))
        return r;
    if (!levels && !gr) {
        // the plain step in fewer launches: HC + FG + the next HC's momentum
        // sum in one kernel, the second HC fused into the second kick's
        // reduction (the kick sees only position differences; in mixed
        // precision the binary64 refinement of cancelling rows, which runs
        // after that reduction, sees the shifted positions)
        const int64_t nsum = hc_count(b, p);
        if ((e = launch_momentum(b, L, (char *)ws, s, nsum)) != hipSuccess) return hip_fail(e);
        if ((e = launch_hc_drift(b, p->m_star, h, p->G * p->m_star, p->dt, L, (char *)ws, s,
                                 nsum)) != hipSuccess)
            return hip_fail(e);
        if ((r = do_kick(b, p, h, nullptr, nullptr, nullptr, nullptr, true, ws, stream, 2, true)))
            return r;
        if (p->flags & GENGA_FLAG_NOSYNC) return GENGA_OK;
        return genga_read_status(ws, stream);
    }
    if (gr && (e = launch_gr(b, p, h, L, (char *)ws, s)) != hipSuccess) return hip_fail(e);
    if ((e = launch_hc(b, p->m_star, h, L, (char *)ws, s, hc_count(b, p))) != hipSuccess)
        return hip_fail(e);
    if (levels && (e = levels_before_drift(b, V, pairs, (char *)ws, s)) != hipSuccess)
        return hip_fail(e);
    if ((e = launch_drift(b, p->G * p->m_star, p->dt, (char *)ws, s)) != hipSuccess)
        return hip_fail(e);
    if (levels && (e = levels_after_drift(b, p, V, (char *)ws, s)) != hipSuccess)
        return hip_fail(e);
    if ((e = launch_hc(b, p->m_star, h, L, (char *)ws, s, hc_count(b, p))) != hipSuccess)
        return hip_fail(e);
    if (gr && (e = launch_gr(b, p, h, L, (char *)ws, s)) != hipSuccess) return hip_fail(e);
    if ((r = do_kick(b, p, h, nullptr, nullptr, nullptr, nullptr, true, ws, stream, 2))) return r;
    if (p->flags & GENGA_FLAG_NOSYNC) return GENGA_OK;
    return genga_read_status(ws, stream);
}

int genga_gr_kick(genga_bodies *b, const genga_params *p, double h, void *ws, void *stream)
{
    int r = check_bodies(b, true, false);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (!ws || !is_fin(h) || !(p->c_light > 0.0)) return GENGA_E_INVAL;
    if (p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    const Layout L = make_layout(b->n, choose_kick_cfg(b->n, p));
    hipError_t e = launch_gr(b, p, h, L, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_collisions(int64_t n, const genga_params *p, void *ws, int64_t *count, int32_t *i,
                     int32_t *j, double *du, int64_t cap, void *stream)
{
    int r = check_params(p);
    if (r) return r;
    if (n < 1 || !ws || !count || !p->direct || cap < 0) return GENGA_E_INVAL;
    if (cap > 0 && (!i || !j || !du)) return GENGA_E_INVAL;
    const LevelLayout V = make_level_layout(n, p, make_layout(n, choose_kick_cfg(n, p)).total);
    hipStream_t s = (hipStream_t)stream;
    uint64_t c = 0;
    hipError_t e = hipMemcpyAsync(&c, (char *)ws + V.coll_count, sizeof(c), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    *count = (int64_t)c;
    const int64_t k = std::min<int64_t>(std::min<int64_t>((int64_t)c, LEVEL_COLL_CAP), cap);
    if (k <= 0) return GENGA_OK;
    std::vector<int32_t> ci(k), cj(k);
    std::vector<double> cd(k);
    e = hipMemcpyAsync(ci.data(), (char *)ws + V.coll_i, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cj.data(), (char *)ws + V.coll_j, sizeof(int32_t) * k,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cd.data(), (char *)ws + V.coll_du, sizeof(double) * k,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    std::vector<int64_t> ord(k);
    for (int64_t q = 0; q < k; ++q) ord[q] = q;
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
        return ci[a] != ci[b] ? ci[a] < ci[b] : cj[a] < cj[b];
    });
    for (int64_t q = 0; q < k; ++q) {
        i[q] = ci[ord[q]];
        j[q] = cj[ord[q]];
        du[q] = cd[ord[q]];
    }
    return GENGA_OK;
}

int genga_group_stats(int64_t n, const genga_params *p, void *ws, int64_t *out, void *stream)
{
    int r = check_params(p);
    if (r) return r;
    if (n < 1 || !ws || !out || !p->direct) return GENGA_E_INVAL;
    const LevelLayout V = make_level_layout(n, p, make_layout(n, choose_kick_cfg(n, p)).total);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(out, (char *)ws + V.gstats, 2 * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_level_counts(int64_t n, const genga_params *p, void *ws, int64_t *out, void *stream)
{
    int r = check_params(p);
    if (r) return r;
    if (n < 1 || !ws || !out || (p->slevels < 2 && !p->direct)) return GENGA_E_INVAL;
    const LevelLayout V = make_level_layout(n, p, make_layout(n, choose_kick_cfg(n, p)).total);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(out, (char *)ws + V.lcount, sizeof(int64_t) * V.L,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

int genga_kick_static(const genga_bodies *b, const genga_params *p, double h, double *ax,
                      double *ay, double *az, genga_pairs *pairs, int32_t *status, void *stream)
{
    int r = check_bodies(b, h != 0.0, true);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if ((r = check_pairs(pairs))) return r;
    if (!status || !is_fin(h)) return GENGA_E_INVAL;
    if ((ax || ay || az) && !(ax && ay && az)) return GENGA_E_INVAL;
    if ((r = check_tp(b, p, true))) return r;
    if (make_layout(b->n, choose_kick_cfg(b->n, p)).total > (size_t)GENGA_STATIC_SCRATCH_BYTES)
        return GENGA_E_SCRATCH;
    void *ws = nullptr;
    if ((r = static_scratch(&ws))) return r;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_static_begin, dim3(1), dim3(64), 0, s, (int32_t *)ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    if ((r = do_kick(b, p, h, ax, ay, az, pairs, true, ws, stream))) return r;
    hipLaunchKernelGGL(k_static_end, dim3(1), dim3(1), 0, s, (const int32_t *)ws, status);
    e = hipGetLastError();
    return e == hipSuccess ? GENGA_OK : hip_fail(e);
}

}  // extern "C"
