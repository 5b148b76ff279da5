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
    ST_NOCONV = 8,     // Kepler solve did not converge
};

constexpr int KB = 256;      // threads per kick block (4 waves of 64)
constexpr int TILE = 256;    // columns staged in LDS per pass
constexpr int WSEG = 128;    // staged encounter pairs per kick wave
constexpr int RB = 256;      // rows per block of the O(N) kernels

// Launch shape of the kick for a system of n bodies.
struct KickCfg {
    int ipt = 1;              // rows per thread
    int slices = 1;           // column slices (grid.y)
    int64_t slice_len = 0;    // columns per slice, a multiple of TILE
    int gx = 0;               // row blocks (grid.x)
    int64_t nwaves = 0;       // kick waves in one launch
};

// Byte offsets of the workspace regions.
struct Layout {
    size_t status = 0;   // int32 status word (+ padding)
    size_t part = 0;     // double [slices][3][npad]  partial accelerations
    size_t cnt = 0;      // int32  [slices][npad]     per-slice pair counts
    size_t rowloc = 0;   // int32  [npad]             row offset inside its 256-row block
    size_t bsum = 0;     // int64  [nb + 1]           per-block pair counts / offsets
    size_t stage = 0;    // int32  [nwaves][WSEG][3]  staged (i, j, rank)
    size_t wcount = 0;   // int32  [nwaves]           staged pairs per wave
    size_t hc = 0;       // double [nb][3]            momentum partials
    size_t total = 0;
    int64_t npad = 0;
    int64_t nb = 0;
};

KickCfg choose_kick_cfg(int64_t n, const genga_params *p);
Layout make_layout(int64_t n, const KickCfg &c);

void set_hip_error(hipError_t e);

// Kernel launchers (return hipError_t of the launch).
struct KickLaunch {
    const double *x, *y, *z, *m, *rc;
    double *vx, *vy, *vz;      // updated when h != 0
    double *ax, *ay, *az;      // optional outputs
    int64_t n;
    double G, h;
    int precision;
    bool forces;               // false: encounter list only
    genga_pairs *pairs;        // optional
    void *ev0, *ev1;           // optional timing events around the main kernel
};
hipError_t launch_kick(const KickLaunch &k, const KickCfg &c, const Layout &L, char *ws,
                       hipStream_t s);

hipError_t launch_rcrit(const genga_bodies *b, const genga_params *p, char *ws, hipStream_t s);
hipError_t launch_hc(genga_bodies *b, double m_star, double h, const Layout &L, char *ws,
                     hipStream_t s);
hipError_t launch_drift(genga_bodies *b, double mu, double dt, char *ws, hipStream_t s);
hipError_t launch_clear_status(char *ws, hipStream_t s);

}  // namespace genga
