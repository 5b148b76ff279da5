// Internal declarations of libgenga.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "genga.h"

namespace genga {

// Bits of the device status word (first int32 of the workspace).
enum : int32_t {
    ST_OVERFLOW = 1,   // encounter list longer than its capacity
    ST_NONFINITE = 2,  // coincident distinct bodies or a non-finite result
    ST_RCRIT = 4,      // negative or NaN critical radius
    ST_NOCONV = 8,     // Kepler solve or Bulirsch-Stoer did not converge
    ST_GROUP = 16,     // a close-encounter group larger than GENGA_GROUP_MAX
};

constexpr int KB = 256;      // threads per kick block (4 waves of 64)
constexpr int WSEG = 128;    // staged encounter pairs per kick wave
constexpr int RB = 256;      // rows per block of the O(N) kernels

// One kick tile: rows [row0, row0 + nrows) of one system against its columns
// [col0, col0 + ncols); `slice` numbers the column ranges of that system.
struct TileDesc {
    int64_t row0;
    int32_t nrows;
    int32_t slice;
    int64_t col0;
    int32_t ncols;
    int32_t sys;
};

// Symmetric binary64 kick of one system (each unordered pair evaluated once,
// its force applied to both bodies).  Rows are cut into groups of SYM_RG (one
// block of SYM_NW waves, SYM_IPT rows per lane); group g works on the columns
// [g SYM_RG, n) in slices of W columns (W divides SYM_RG, d = SYM_RG / W of
// them cover the group's own rows).  A tile is (group g, slice s), stored as
// sid = tb(g) + s; launched as the d..ns(g)-1 slices of every group first,
// then the d diagonal slices of every group.
constexpr int SYM_NW = 4;
constexpr int SYM_IPT = 2;
constexpr int SYM_NT = SYM_NW * 64;
constexpr int SYM_RG = SYM_NT * SYM_IPT;

struct SymShape {
    int64_t n = 0;
    int64_t G = 0;       // row groups
    int64_t S0 = 0;      // slices of group 0 (ceil(n / W))
    int W = 0, d = 0;    // columns per slice, slices over a group's own rows
    int64_t T = 0;       // tiles
    int64_t tfull = 0;   // tiles off the diagonal (launched first)
    // slices of group g, first storage tile of group g
    __host__ __device__ int64_t ns(int64_t g) const { return S0 - g * d; }
    __host__ __device__ int64_t tb(int64_t g) const { return g * S0 - d * ((g * (g - 1)) / 2); }
    // column sums of group g: 3 rows of collen(g) doubles from 3 coloff(g)
    __host__ __device__ int64_t collen(int64_t g) const { return n - g * SYM_RG; }
    __host__ __device__ int64_t coloff(int64_t g) const
    {
        return g * n - (int64_t)SYM_RG * ((g * (g - 1)) / 2);
    }
    // tiles off the diagonal before group g
    __host__ __device__ int64_t bf(int64_t g) const { return g * S0 - d * ((g * (g + 1)) / 2); }
};
SymShape sym_shape(int64_t n, int W);

// Batch of systems in the symmetric kick: per system its shape (n = its
// bodies), first body o, first storage tile tbase and the offset cbase of
// its column sums (in doubles, per component block as in one system); per
// tile (in storage order) its system, group and slice; order[t] the storage
// number of the t-th launched tile (decreasing work).
struct SymSys {
    SymShape sh;
    int64_t o, tbase, cbase;
};
struct SymTileB {
    int32_t sys, g, s, pad;
};
struct SymBatch {
    const SymSys *sys;
    const SymTileB *tiles;
    const int32_t *order;
    int64_t S, T;
};
constexpr int64_t SYM_MIN_N = 8192;    // default: symmetric kick from this many bodies
// below this many bodies the symmetric kick's row totals are summed in
// SYM_FOLD parts over the whole chip before the reduction (k_sym_fold)
constexpr int64_t SYM_FOLD_BELOW = 32768;
// default limit of the symmetric kick's row and column sums (about 370,000
// bodies); larger systems take the one-sided form unless forced
constexpr int64_t SYM_WS_MAX = (int64_t)8 << 30;
constexpr int SYM_FOLD = 8;
hipError_t launch_kick_sym(const SymShape &h, bool mixed, double widen, const double *x,
                           const double *y, const double *z, const double *m, const double *rc,
                           double *rowpart, double *colpart, int32_t *cnt, int32_t *stage,
                           int32_t *wcount, int32_t *status, int32_t *refine_cnt, bool emit,
                           hipStream_t s);
hipError_t launch_kick_vjp_sym(const SymShape &h, const genga_bodies *b, double G, double scale,
                               const double *abx, const double *aby, const double *abz,
                               genga_adjoint *adj, double *part, int32_t *status, hipStream_t s);
hipError_t launch_kick_sym_b(const SymBatch &b, const double *x, const double *y,
                             const double *z, const double *m, const double *rc, double *rowpart,
                             double *colpart, int32_t *cnt, int32_t *stage, int32_t *wcount,
                             int32_t *status, bool emit, hipStream_t s);
hipError_t launch_scatter_sym(const SymShape &h, const SymBatch *b, const double *x,
                              const double *y, const double *z, const double *rc,
                              const int32_t *cnt, const int32_t *stage, const int32_t *wcount,
                              const int32_t *rowloc, const int64_t *boff, genga_pairs *pairs,
                              hipStream_t s);

// Launch shape of the kick.
struct KickCfg {
    int nt = KB;              // threads per block (64 or 256)
    int ipt = 1;              // rows per thread
    int slices = 1;           // column slices (single system: grid.y; batch: max per system)
    int64_t slice_len = 0;    // single system: columns per slice, a multiple of 64
    int gx = 0;               // single system: row blocks (grid.x)
    int64_t ntiles = 0;       // tiles in one launch
    int64_t nwaves = 0;       // kick waves in one launch (ntiles * nt / 64)
    int grid = 0;             // batch: persistent blocks
    int gy = 0;               // single system: grid.y of the launch (grid.x = gx)
    // single system in a test-particle mode (tp = 1 or 2): rows [0, nm) are
    // the massive bodies (gx_m row blocks, s_m slices of len_m over all
    // columns), rows [nm, n) the test particles (gx_t row blocks, s_t slices
    // of len_t over the massive columns); tiles are numbered massive first.
    // The massive rows' partial sums form a compact block [s_m][.][mpad]
    // ahead of the test particles' [s_t][.][npad]; slices then counts the
    // npad-long slice rows that both need (it sizes the workspace).
    int tp = 0;
    int64_t nm = 0;
    int gx_m = 0, s_m = 0, gx_t = 0, s_t = 0;
    int64_t len_m = 0, len_t = 0;
    int64_t mpad = 0;
    // binary64 forces of one system: the symmetric kick (sym.T > 0) instead
    // of the one-sided tiles above
    bool use_sym = false;
    SymShape sym;
    // binary64 batch in the symmetric kick: tiles and column-sum doubles (per
    // component) of all systems
    bool use_symb = false;
    int64_t symb_S = 0, symb_T = 0, symb_cols = 0;
    int symb_W = 0;           // columns per slice of every system (512, 256 or 128)
};

// Byte offsets of the workspace regions.
struct Layout {
    size_t status = 0;     // int32 status word, tile counter, refine count (+ padding)
    size_t part = 0;       // double [slices][5][npad]  partial sums (kick: 3, adjoint: 5)
    size_t cnt = 0;        // int32  [slices][npad]     per-slice pair counts
    size_t rowloc = 0;     // int32  [npad]             row offset inside its 256-row block
    size_t bsum = 0;       // int64  [nb + 1]           per-block pair counts / offsets
    size_t stage = 0;      // int32  [nwaves][WSEG][3]  staged (i, j, rank)
    size_t wcount = 0;     // int32  [nwaves]           staged pairs per wave
    size_t hc = 0;         // double [nb][3]            momentum partials
    size_t hc2 = 0;        // double [nb][3]            momentum partials (second buffer)
    size_t rlist = 0;      // int32  [npad]             mixed: rows to evaluate in binary64
    size_t gru = 0;        // double [3][npad]          post-Newtonian: new heliocentric velocities
    size_t grp = 0;        // double [nb][4]            post-Newtonian: partial sums of m u', m
    size_t P = 0;          // batch: double [S][3]      momentum per system
    size_t tiles = 0;      // batch: TileDesc [ntiles]
    size_t sysid = 0;      // batch: int32 [npad]
    size_t sys_slices = 0; // batch: int32 [S]
    size_t offsets = 0;    // batch: int64 [S + 1]
    size_t symsys = 0;     // batch, symmetric kick: SymSys [S]
    size_t symtiles = 0;   // batch, symmetric kick: SymTileB [T]
    size_t symorder = 0;   // batch, symmetric kick: int32 [T]
    size_t total = 0;
    int64_t npad = 0;
    int64_t nb = 0;
};

KickCfg choose_kick_cfg(int64_t n, const genga_params *p);
// Resident blocks per CU of the persistent kick for this shape (0 if unknown).
int kick_blocks_per_cu(const KickCfg &c, int precision);
Layout make_layout(int64_t n, const KickCfg &c, int64_t S = 0);

void set_hip_error(hipError_t e);

// Kernel launchers (return hipError_t of the launch).
struct KickLaunch {
    const double *x, *y, *z, *m, *rc;
    double *vx, *vy, *vz;      // updated when the step factor is non-zero
    double *ax, *ay, *az;      // optional outputs
    int64_t n;
    double G, h;               // single system: v += h a
    double hfac;               // batch: v += hfac * dt_s * a
    int precision;
    bool forces;               // false: encounter list only
    genga_pairs *pairs;        // optional
    void *ev0, *ev1;           // optional timing events around the main kernel
    const TileDesc *tiles;     // batch: device tile list (else null)
    const int32_t *sysid;      // batch: system of each body
    const int32_t *sys_slices; // batch: column slices per system
    const double *sys_dt;      // batch: time step per system
    const int64_t *sys_off;    // batch: device offsets of the systems
    // optional: after the velocities, x += hc_h P / hc_m_star for every body,
    // P the fixed-order sum of the hc_nb momentum partials hc_part (the Sun
    // kick H_C fused into the reduction; the kick itself only sees
    // differences of positions, which a common shift leaves unchanged)
    double *px = nullptr, *py = nullptr, *pz = nullptr;
    const double *hc_part = nullptr;
    int64_t hc_nb = 0;
    double hc_h = 0.0, hc_m_star = 1.0;
};
hipError_t launch_kick(const KickLaunch &k, const KickCfg &c, const Layout &L, char *ws,
                       hipStream_t s);

hipError_t launch_rcrit(const genga_bodies *b, const genga_params *p, char *ws, hipStream_t s);
// x_i += h P / m_star for every body, P summed over bodies [0, nsum).
hipError_t launch_hc(genga_bodies *b, double m_star, double h, const Layout &L, char *ws,
                     hipStream_t s, int64_t nsum);
hipError_t launch_drift(genga_bodies *b, double mu, double dt, char *ws, hipStream_t s);
// Momentum partials of bodies [0, nsum) into L.hc.
hipError_t launch_momentum(const genga_bodies *b, const Layout &L, char *ws, hipStream_t s,
                           int64_t nsum);
// HC(h) with the partials in L.hc, the drift FG(dt), and the momentum
// partials of the drifted velocities (bodies [0, nsum)) into L.hc2: one kernel.
hipError_t launch_hc_drift(genga_bodies *b, double m_star, double h, double mu, double dt,
                           const Layout &L, char *ws, hipStream_t s, int64_t nsum);
hipError_t launch_gr(genga_bodies *b, const genga_params *p, double h, const Layout &L, char *ws,
                     hipStream_t s);
hipError_t launch_clear_status(char *ws, hipStream_t s);
hipError_t launch_energy(const genga_bodies *b, const genga_params *p, double *out,
                         const KickCfg &c, const Layout &L, char *ws, hipStream_t s);
// out[5] = out[0] + the changeover-potential correction over the listed pairs.
hipError_t launch_energy_k_pairs(const genga_bodies *b, const genga_params *p, genga_pairs *pairs,
                                 double *out, const Layout &L, char *ws, hipStream_t s);

// Device view of a planned batch (pointers into the caller's arrays and the
// workspace).
struct BatchDev {
    int64_t S;
    const int64_t *offsets;     // device, S + 1 (workspace copy)
    const int32_t *sysid;       // device, per body
    const int32_t *sys_slices;  // device, per system
    const TileDesc *tiles;      // device tile list
    const double *m_star, *dt, *n1, *n2;  // caller's device arrays
    double *P;                  // workspace: momentum per system (S x 3)
};
hipError_t launch_kick_vjp(const genga_bodies *b, const genga_params *p, double scale,
                           const double *abx, const double *aby, const double *abz,
                           genga_adjoint *adj, char *ws, hipStream_t s);
hipError_t launch_rcrit_vjp(const genga_bodies *b, const genga_params *p, genga_adjoint *adj,
                            hipStream_t s);
hipError_t launch_hc_vjp(const genga_bodies *b, const genga_params *p, double h, genga_adjoint *adj,
                         const Layout &L, char *ws, hipStream_t s);
hipError_t launch_drift_vjp(const genga_bodies *b, const genga_params *p, double dt,
                            genga_adjoint *adj, char *ws, hipStream_t s);
hipError_t launch_rcrit_b(const genga_bodies *b, const BatchDev &bd, char *ws, hipStream_t s);
hipError_t launch_hc_b(genga_bodies *b, const BatchDev &bd, double hfac, hipStream_t s);
hipError_t launch_drift_b(genga_bodies *b, const BatchDev &bd, double G, double hfac, char *ws,
                          hipStream_t s);

// Symplectic levels (genga_step with slevels > 1): workspace regions placed
// after the kick's Layout.  Lists l = 0 .. L-1 (E_0 from the first half kick,
// E_l detected at level l); adjacency, body list and saved states for the
// lists that a deeper level integrates (l = 0 .. L-2); critical radii of the
// levels 1 .. L-1 (level 0 uses the bodies' rc).
struct LevelLayout {
    int L = 0;
    int64_t cap = 0;
    size_t lcount = 0;                  // int64 [L]   summed list sizes per level
    size_t cnt = 0;                     // int64 [L]   current size of list l
    size_t nbod = 0;                    // int32 [L]   bodies of list l
    size_t bcnt = 0;                    // int64 [DB]  detection block counts / offsets
    size_t tsum = 0;                    // int64 [2][n / 256] adjacency tile sums / offsets
    size_t pi[GENGA_MAX_LEVELS] = {}, pj[GENGA_MAX_LEVELS] = {};   // int32 [cap]
    size_t start[GENGA_MAX_LEVELS] = {};   // int32 [n + 1]  adjacency offsets
    size_t adj[GENGA_MAX_LEVELS] = {};     // int32 [2 cap]  partners, ascending per body
    size_t adj_tmp[GENGA_MAX_LEVELS] = {}; // int32 [2 cap]  partners in arrival order
    size_t owner[GENGA_MAX_LEVELS] = {};   // int32 [2 cap]  body of each arrival entry
    size_t deg[GENGA_MAX_LEVELS] = {};     // int32 [n]      degrees / fill counters
    size_t bodies[GENGA_MAX_LEVELS] = {};  // int32 [n]      bodies of the list, ascending
    size_t rc[GENGA_MAX_LEVELS] = {};      // double [n]     rc of level l (l >= 1)
    size_t shadow[GENGA_MAX_LEVELS] = {};  // double [6][n]  state saved before a drift
    // direct solver (groups of the deepest list L - 1)
    int direct = 0;
    size_t glab = 0;       // int32 [n]  parent in the union-find, then the group's root
    size_t gflag = 0;      // int32 [n]  body in the deepest list
    size_t gsize = 0;      // int32 [n]  members per root
    size_t gfill = 0;      // int32 [n]  fill counters per root
    size_t gstart = 0;     // int32 [n]  first member slot per root
    size_t groot = 0;      // int32 [n]  roots in ascending order (one per group)
    size_t gtmp = 0;       // int32 [n]  members in arrival order
    size_t gmem = 0;       // int32 [n]  members, ascending within each group of <= 512
    size_t gcount = 0;     // int32 [2]  groups, members
    size_t gstats = 0;     // int64 [2]  groups integrated, largest group (per step)
    size_t gtsum = 0;      // int64 [2][n / 256] tile sums of the group scan
    size_t coll_count = 0; // uint64     collisions of the step
    size_t coll_i = 0, coll_j = 0;   // int32 [LEVEL_COLL_CAP] survivor, absorbed
    size_t coll_du = 0;    // double [LEVEL_COLL_CAP] lost energy
    // grid solver (groups of more than 512 bodies; n > 512 only): capacity
    // gcap = min(n rounded up to 256, GENGA_GROUP_MAX) members
    int64_t gcap = 0;
    size_t gbig = 0;       // int32 [2 + n / 513]  listed groups, their roots
    size_t gsync = 0;      // uint64 [8]  barrier arrivals, abort, reduction slots
    size_t gpub = 0;       // double [2][6][gcap]  published member states
    size_t gbox = 0;       // double [2][gcap / 64][8]  tile boxes
    size_t gtrho = 0;      // double [gcap / 64]  largest deepest-level rc per tile
    size_t gmm = 0, gmR = 0, gmrc = 0;   // double [gcap]  mass, radius, deepest rc
    size_t gmirc = 0;      // double [L][gcap]  1 / rc per level
    size_t gmidx = 0;      // int32 [gcap]  member bodies
    size_t gbpart = 0;     // double [gcap / 64][4]  workgroup extents
    size_t gccnt = 0, gcfill = 0;   // int32 [4096]  ordering cells
    size_t gctmp = 0;      // int32 [2][gcap]  cell scratch, spatial order
    size_t total = 0;
};

constexpr int64_t LEVEL_COLL_CAP = 4096;   // collision records kept per step
// base: byte offset where the level regions start (the kick Layout's total).
LevelLayout make_level_layout(int64_t n, const genga_params *p, size_t base);
// The level-0 list in the workspace (the first half kick writes it there).
genga_pairs level0_pairs(const LevelLayout &V, char *ws);
// After the first half kick and HC: record |E_0|, copy E_0 to the caller's
// list (nullable), build its adjacency and save its bodies' state.
hipError_t levels_before_drift(const genga_bodies *b, const LevelLayout &V, genga_pairs *out,
                               char *ws, hipStream_t s);
// After the drift of every body: restore E_0's bodies and run levels 1 .. L-1
// (with the direct solver: for L = 1 the groups of E_0, else those of each
// sub-step of level L - 1).
hipError_t levels_after_drift(genga_bodies *b, const genga_params *p, const LevelLayout &V,
                              char *ws, hipStream_t s);

}  // namespace genga
