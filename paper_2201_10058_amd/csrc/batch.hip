// Batched ensembles: many independent systems of uneven size in one
// persistent kick launch.  The paper names a multi-simulation mode (Sect. 10)
// without describing it; here each system is an independent instance of the
// base step of Appendix A and the systems share one launch per operator.
//
// Host side: a plan (tile list sorted by cost, body -> system map, column
// slices per system) is written into the caller's workspace once; the
// batched kick then walks that list with a persistent grid, so a step is a
// fixed sequence of launches that can be captured in one hipGraph.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <mutex>
#include <queue>
#include <unordered_map>
#include <vector>

#include "genga_internal.h"

namespace genga {

static int cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

struct BatchShape {
    KickCfg cfg;
    int64_t ntot = 0;
    int64_t cols = 0;     // columns per tile (multiple of 64)
};

// Symmetric kick of a batch: the critical path of one tile, in units of one
// 64-row slot's pass over a 64-column chunk.  At each chunk the block waits
// for its busiest wave: off the diagonal both slots of every wave run the
// chunk (padding rows included); on a diagonal tile a slot works on the
// chunks from its own on and padding slots are skipped.  Each chunk and each
// tile also carry a fixed cost (staging, barriers, sums).
static double sym_tile_cost(const SymShape &h, int64_t g, int64_t s)
{
    const int64_t row0 = g * SYM_RG;
    const int64_t rowend = std::min<int64_t>(row0 + SYM_RG, h.n);
    const int64_t col0 = row0 + s * h.W;
    const int64_t col1 = std::min<int64_t>(col0 + h.W, h.n);
    const int64_t nch = (col1 - col0 + 63) / 64;
    double t = 0.5;
    for (int64_t kc = 0; kc < nch; ++kc) {
        const int64_t cc = (col0 >> 6) + kc;
        int busiest = 0;
        for (int w = 0; w < SYM_NW; ++w) {
            int c = 0;
            for (int q = 0; q < SYM_IPT; ++q) {
                const int64_t slot = (int64_t)q * SYM_NW + w;
                if (s >= h.d) {
                    ++c;
                } else if (row0 + slot * 64 < rowend && cc >= (row0 >> 6) + slot) {
                    ++c;
                }
            }
            busiest = std::max(busiest, c);
        }
        t += busiest + 0.15;
    }
    return t;
}

// Longest total, over the resident blocks, of the tiles handed out in
// decreasing cost as blocks free up (the launch's order and schedule).
static double sym_makespan(std::vector<double> &cost, int slots)
{
    std::sort(cost.begin(), cost.end(), std::greater<double>());
    std::priority_queue<double, std::vector<double>, std::greater<double>> q;
    for (int k = 0; k < slots; ++k) q.push(0.0);
    for (double c : cost) {
        const double m = q.top();
        q.pop();
        q.push(m + c);
    }
    double mx = 0.0;
    while (!q.empty()) {
        mx = std::max(mx, q.top());
        q.pop();
    }
    return mx;
}

// Columns per slice for a batch in the symmetric kick: of 512, 256 and 128
// (one, two or four slices per 512-row group), the width whose tiles finish
// first on the device's resident blocks by the model above (narrower slices
// balance the blocks better but add tiles and row sums).  The 512-system
// ensemble of 16-4,096 bodies takes 256 (0.803 against 0.839 ms per step
// for 512 and 0.834 for 128).
static int sym_batch_width_uncached(const genga_batch *bt, int slots)
{
    int best = SYM_RG;
    double best_t = 0.0;
    for (int W : {SYM_RG, SYM_RG / 2, SYM_RG / 4}) {
        std::vector<double> cost;
        for (int64_t q = 0; q < bt->S; ++q) {
            const SymShape h = sym_shape(bt->offsets[q + 1] - bt->offsets[q], W);
            for (int64_t g = 0; g < h.G; ++g)
                for (int64_t k = 0; k < h.ns(g); ++k) cost.push_back(sym_tile_cost(h, g, k));
        }
        const double t = sym_makespan(cost, slots);
        if (W == SYM_RG || t < best_t) {
            best = W;
            best_t = t;
        }
    }
    return best;
}

// The same, remembered per (system sizes, resident blocks): the simulation
// takes tens of microseconds of host time, and every batched call derives
// its shape again.
static int sym_batch_width(const genga_batch *bt)
{
    const int slots = 4 * cu_count();   // blocks of 4 waves at 4 waves per SIMD
    uint64_t h = 1469598103934665603ull ^ (uint64_t)slots;
    for (int64_t q = 0; q <= bt->S; ++q) h = (h ^ (uint64_t)bt->offsets[q]) * 1099511628211ull;
    static std::mutex mu;
    static std::unordered_map<uint64_t, int> memo;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(h);
        if (it != memo.end()) return it->second;
    }
    const int W = sym_batch_width_uncached(bt, slots);
    std::lock_guard<std::mutex> lk(mu);
    if (memo.size() > 4096) memo.clear();
    memo[h] = W;
    return W;
}

// Validate the batch and derive the launch shape (O(S) host work).
static int batch_shape(const genga_batch *bt, const genga_params *p, BatchShape &sh)
{
    if (!bt || bt->S < 1 || !bt->offsets) return GENGA_E_INVAL;
    if (!bt->m_star || !bt->dt || !bt->n1 || !bt->n2) return GENGA_E_INVAL;
    if (bt->offsets[0] != 0) return GENGA_E_INVAL;
    if (p && p->tp_mode != 0) return GENGA_E_UNSUPPORTED;
    KickCfg &c = sh.cfg;
    c.nt = (p && p->block == 64) ? 64 : KB;
    if (p && p->block != 0 && p->block != 64 && p->block != KB) return GENGA_E_INVAL;
    c.ipt = (p && p->ipt > 0) ? p->ipt : 1;
    if (c.ipt != 1 && c.ipt != 2) return GENGA_E_INVAL;
    int64_t cols = (p && p->tile_cols > 0) ? p->tile_cols : 1024;
    cols = ((cols + 63) / 64) * 64;
    sh.cols = cols;
    const int64_t R = (int64_t)c.nt * c.ipt;
    int64_t ntiles = 0;
    int maxs = 1;
    for (int64_t s = 0; s < bt->S; ++s) {
        const int64_t ns = bt->offsets[s + 1] - bt->offsets[s];
        if (ns < 1) return GENGA_E_INVAL;
        const int64_t rb = (ns + R - 1) / R;
        const int64_t nsl = (ns + cols - 1) / cols;
        ntiles += rb * nsl;
        if (nsl > maxs) maxs = (int)nsl;
    }
    sh.ntot = bt->offsets[bt->S];
    if (sh.ntot > (int64_t)INT32_MAX) return GENGA_E_INVAL;
    c.slices = maxs;
    c.ntiles = ntiles;
    c.nwaves = ntiles * (c.nt / 64);
    int per_cu = kick_blocks_per_cu(c, p ? p->precision : GENGA_FP64);
    if (per_cu <= 0) per_cu = c.nt == 64 ? 8 : 2;
    int64_t grid = (p && p->grid > 0) ? p->grid : (int64_t)cu_count() * per_cu;
    if (grid > ntiles) grid = ntiles;
    c.grid = (int)grid;
    // binary64: the symmetric kick over every system (512-row groups and
    // slices of symb_W columns, the same width for every system)
    if ((!p || p->precision == GENGA_FP64) && !(p && (p->flags & GENGA_FLAG_DIRECTED))) {
        const int sl = p ? p->slices : 0;
        if (sl < 0) return GENGA_E_INVAL;
        int d = 1;
        while (2 * d <= sl && 2 * d <= 4) d *= 2;
        c.use_symb = true;
        c.symb_W = sl ? SYM_RG / d : sym_batch_width(bt);
        c.symb_S = bt->S;
        c.symb_T = 0;
        c.symb_cols = 0;
        for (int64_t q = 0; q < bt->S; ++q) {
            const SymShape h = sym_shape(bt->offsets[q + 1] - bt->offsets[q], c.symb_W);
            c.symb_T += h.T;
            c.symb_cols += h.coloff(h.G);
        }
    }
    return GENGA_OK;
}

// Symmetric kick of a batch: per-system shapes and offsets, tiles in storage
// order (system by system, tb(g) + s within a system) and the launch order
// (decreasing critical path, sym_tile_cost).
static void build_sym_plan(const genga_batch *bt, const BatchShape &sh, std::vector<SymSys> &sys,
                           std::vector<SymTileB> &tiles, std::vector<int32_t> &order)
{
    sys.assign((size_t)bt->S, SymSys{});
    tiles.clear();
    tiles.reserve((size_t)sh.cfg.symb_T);
    std::vector<double> cost;
    cost.reserve((size_t)sh.cfg.symb_T);
    int64_t tbase = 0, cbase = 0;
    for (int64_t q = 0; q < bt->S; ++q) {
        SymSys &ss = sys[(size_t)q];
        ss.o = bt->offsets[q];
        ss.sh = sym_shape(bt->offsets[q + 1] - ss.o, sh.cfg.symb_W);
        ss.tbase = tbase;
        ss.cbase = cbase;
        for (int64_t g = 0; g < ss.sh.G; ++g) {
            for (int64_t k = 0; k < ss.sh.ns(g); ++k) {
                tiles.push_back(SymTileB{(int32_t)q, (int32_t)g, (int32_t)k, 0});
                cost.push_back(sym_tile_cost(ss.sh, g, k));
            }
        }
        tbase += ss.sh.T;
        cbase += 3 * ss.sh.coloff(ss.sh.G);
    }
    order.resize(tiles.size());
    for (size_t t = 0; t < order.size(); ++t) order[t] = (int32_t)t;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cost[(size_t)a] > cost[(size_t)b]; });
}

// Tile list (sorted by decreasing work, ties by position), body -> system map
// and column slices per system.
static void build_plan(const genga_batch *bt, const BatchShape &sh, std::vector<TileDesc> &tiles,
                       std::vector<int32_t> &sysid, std::vector<int32_t> &slices)
{
    const int64_t R = (int64_t)sh.cfg.nt * sh.cfg.ipt;
    tiles.clear();
    tiles.reserve((size_t)sh.cfg.ntiles);
    sysid.assign((size_t)sh.ntot, 0);
    slices.assign((size_t)bt->S, 0);
    for (int64_t s = 0; s < bt->S; ++s) {
        const int64_t off = bt->offsets[s];
        const int64_t ns = bt->offsets[s + 1] - off;
        const int64_t nsl = (ns + sh.cols - 1) / sh.cols;
        slices[(size_t)s] = (int32_t)nsl;
        for (int64_t i = 0; i < ns; ++i) sysid[(size_t)(off + i)] = (int32_t)s;
        for (int64_t r0 = 0; r0 < ns; r0 += R) {
            for (int64_t k = 0; k < nsl; ++k) {
                TileDesc t;
                t.row0 = off + r0;
                t.nrows = (int32_t)std::min(R, ns - r0);
                t.slice = (int32_t)k;
                t.col0 = off + k * sh.cols;
                t.ncols = (int32_t)std::min(sh.cols, ns - k * sh.cols);
                t.sys = (int32_t)s;
                tiles.push_back(t);
            }
        }
    }
    std::stable_sort(tiles.begin(), tiles.end(), [](const TileDesc &a, const TileDesc &b) {
        return (int64_t)a.nrows * a.ncols > (int64_t)b.nrows * b.ncols;
    });
}

static BatchDev batch_dev(const genga_batch *bt, const Layout &L, char *ws)
{
    BatchDev bd;
    bd.S = bt->S;
    bd.offsets = (const int64_t *)(ws + L.offsets);
    bd.sysid = (const int32_t *)(ws + L.sysid);
    bd.sys_slices = (const int32_t *)(ws + L.sys_slices);
    bd.tiles = (const TileDesc *)(ws + L.tiles);
    bd.m_star = bt->m_star;
    bd.dt = bt->dt;
    bd.n1 = bt->n1;
    bd.n2 = bt->n2;
    bd.P = (double *)(ws + L.P);
    return bd;
}

static int hip_err(hipError_t e)
{
    set_hip_error(e);
    return GENGA_E_HIP;
}

static int kick_batched(const genga_bodies *b, const genga_batch *bt, const genga_params *p,
                        double hfac, double *ax, double *ay, double *az, genga_pairs *pairs,
                        bool forces, void *ws, void *stream, int ev_slot)
{
    BatchShape sh;
    int r = batch_shape(bt, p, sh);
    if (r) return r;
    if (b->n != sh.ntot) return GENGA_E_INVAL;
    const Layout L = make_layout(sh.ntot, sh.cfg, bt->S);
    const BatchDev bd = batch_dev(bt, L, (char *)ws);
    KickLaunch k;
    k.x = b->x; k.y = b->y; k.z = b->z; k.m = b->m; k.rc = b->rc;
    k.vx = b->vx; k.vy = b->vy; k.vz = b->vz;
    k.ax = ax; k.ay = ay; k.az = az;
    k.n = b->n;
    k.G = p->G;
    k.h = 0.0;
    k.hfac = hfac;
    k.precision = p->precision;
    k.forces = forces;
    k.pairs = pairs;
    k.ev0 = p->prof_events[ev_slot];
    k.ev1 = p->prof_events[ev_slot + 1];
    k.tiles = bd.tiles;
    k.sysid = bd.sysid;
    k.sys_slices = bd.sys_slices;
    k.sys_dt = bd.dt;
    k.sys_off = bd.offsets;
    hipError_t e = launch_kick(k, sh.cfg, L, (char *)ws, (hipStream_t)stream);
    return e == hipSuccess ? GENGA_OK : hip_err(e);
}

}  // namespace genga

using namespace genga;

extern "C" {

size_t genga_batch_workspace_bytes(const genga_batch *bt, const genga_params *p)
{
    BatchShape sh;
    if (batch_shape(bt, p, sh)) return 0;
    return make_layout(sh.ntot, sh.cfg, bt->S).total;
}

int genga_batch_plan(const genga_batch *bt, const genga_params *p, void *ws, void *stream)
{
    BatchShape sh;
    int r = batch_shape(bt, p, sh);
    if (r) return r;
    if (!ws) return GENGA_E_INVAL;
    const Layout L = make_layout(sh.ntot, sh.cfg, bt->S);
    std::vector<TileDesc> tiles;
    std::vector<int32_t> sysid, slices;
    build_plan(bt, sh, tiles, sysid, slices);
    char *w = (char *)ws;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if ((e = hipMemcpyAsync(w + L.tiles, tiles.data(), tiles.size() * sizeof(TileDesc),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_err(e);
    if ((e = hipMemcpyAsync(w + L.sysid, sysid.data(), sysid.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_err(e);
    if ((e = hipMemcpyAsync(w + L.sys_slices, slices.data(), slices.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_err(e);
    if ((e = hipMemcpyAsync(w + L.offsets, bt->offsets, (size_t)(bt->S + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_err(e);
    if (sh.cfg.use_symb) {
        std::vector<SymSys> ssys;
        std::vector<SymTileB> stiles;
        std::vector<int32_t> sorder;
        build_sym_plan(bt, sh, ssys, stiles, sorder);
        if ((e = hipMemcpyAsync(w + L.symsys, ssys.data(), ssys.size() * sizeof(SymSys),
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_err(e);
        if ((e = hipMemcpyAsync(w + L.symtiles, stiles.data(), stiles.size() * sizeof(SymTileB),
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_err(e);
        if ((e = hipMemcpyAsync(w + L.symorder, sorder.data(), sorder.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_err(e);
    }
    const int32_t zero2[2] = {0, 0};   // status word and tile counter
    if ((e = hipMemcpyAsync(w + L.status, zero2, sizeof(zero2), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return hip_err(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(e);
    return GENGA_OK;
}

int genga_batch_info(const genga_batch *bt, const genga_params *p, int64_t *out5)
{
    BatchShape sh;
    int r = batch_shape(bt, p, sh);
    if (r) return r;
    if (!out5) return GENGA_E_INVAL;
    out5[0] = sh.cfg.ntiles;
    out5[1] = sh.cfg.grid;
    out5[2] = sh.cfg.nt;
    out5[3] = sh.cfg.ipt;
    out5[4] = sh.cols;
    return GENGA_OK;
}

int genga_kick_batched(const genga_bodies *b, const genga_batch *bt, const genga_params *p,
                       double hfac, double *ax, double *ay, double *az, genga_pairs *pairs,
                       void *ws, void *stream)
{
    if (!b || !b->x || !b->y || !b->z || !b->m || !b->rc || !ws || !p) return GENGA_E_INVAL;
    if (!std::isfinite(hfac) || !std::isfinite(p->G) || p->G < 0.0) return GENGA_E_INVAL;
    if (hfac != 0.0 && (!b->vx || !b->vy || !b->vz)) return GENGA_E_INVAL;
    if ((ax || ay || az) && !(ax && ay && az)) return GENGA_E_INVAL;
    if (pairs && (!pairs->count || pairs->capacity < 0 || (pairs->capacity > 0 && (!pairs->i || !pairs->j))))
        return GENGA_E_INVAL;
    if (p->precision != GENGA_FP64 && p->precision != GENGA_MIXED) return GENGA_E_INVAL;
    if (p->c_light != 0.0 || p->slevels > 1 || p->direct || p->tp_mode != 0)
        return GENGA_E_UNSUPPORTED;
    return kick_batched(b, bt, p, hfac, ax, ay, az, pairs, true, ws, stream, 0);
}

int genga_step_batched(genga_bodies *b, const genga_batch *bt, const genga_params *p,
                       genga_pairs *pairs, void *ws, void *stream)
{
    if (!b || !b->x || !b->y || !b->z || !b->m || !b->rc || !b->vx || !b->vy || !b->vz || !ws || !p)
        return GENGA_E_INVAL;
    if (!std::isfinite(p->G) || p->G < 0.0) return GENGA_E_INVAL;
    if (pairs && (!pairs->count || pairs->capacity < 0 || (pairs->capacity > 0 && (!pairs->i || !pairs->j))))
        return GENGA_E_INVAL;
    if (p->precision != GENGA_FP64 && p->precision != GENGA_MIXED) return GENGA_E_INVAL;
    if (p->c_light != 0.0 || p->slevels > 1 || p->direct || p->tp_mode != 0)
        return GENGA_E_UNSUPPORTED;
    BatchShape sh;
    int r = batch_shape(bt, p, sh);
    if (r) return r;
    if (b->n != sh.ntot) return GENGA_E_INVAL;
    const Layout L = make_layout(sh.ntot, sh.cfg, bt->S);
    const BatchDev bd = batch_dev(bt, L, (char *)ws);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if ((e = launch_rcrit_b(b, bd, (char *)ws, s)) != hipSuccess) return hip_err(e);
    if ((r = kick_batched(b, bt, p, 0.5, nullptr, nullptr, nullptr, pairs, true, ws, stream, 0)))
        return r;
    if ((e = launch_hc_b(b, bd, 0.5, s)) != hipSuccess) return hip_err(e);
    if ((e = launch_drift_b(b, bd, p->G, 1.0, (char *)ws, s)) != hipSuccess) return hip_err(e);
    if ((e = launch_hc_b(b, bd, 0.5, s)) != hipSuccess) return hip_err(e);
    if ((r = kick_batched(b, bt, p, 0.5, nullptr, nullptr, nullptr, nullptr, true, ws, stream, 2)))
        return r;
    if (p->flags & GENGA_FLAG_NOSYNC) return GENGA_OK;
    return genga_read_status(ws, stream);
}

}  // extern "C"
