// Device helpers of the symmetric (rotating-column) kernels: the kick and
// its adjoint.
#pragma once

#include "genga_internal.h"

namespace genga {

// Lane l receives lane (l + 1) mod 64's value.
__device__ __forceinline__ double rotate_down(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x134, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float rotate_down(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xF, 0xF, false));
}

// Tile of launch index t: group g and slice s (s = -1: an empty diagonal slot
// of the last group).
__device__ __forceinline__ void sym_tile(const SymShape &h, int64_t t, int64_t &g, int64_t &s)
{
    if (t < h.tfull) {
        // largest g with bf(g) <= t: root of d/2 g^2 - (S0 - d/2) g + t = 0
        const double b = (double)h.S0 - 0.5 * h.d;
        double r = b * b - 2.0 * h.d * (double)t;
        r = r > 0.0 ? r : 0.0;
        int64_t gg = (int64_t)((b - __builtin_sqrt(r)) / h.d);
        gg = gg < 0 ? 0 : (gg > h.G - 2 ? h.G - 2 : gg);
        while (gg > 0 && h.bf(gg) > t) --gg;
        while (gg < h.G - 2 && h.bf(gg + 1) <= t) ++gg;
        g = gg;
        s = h.d + (t - h.bf(gg));
        return;
    }
    const int64_t u = t - h.tfull;
    g = u / h.d;
    s = u % h.d;
    if (s >= h.ns(g)) s = -1;
}

// Group of storage tile sid: largest g with tb(g) <= sid.
__device__ __forceinline__ int64_t sym_group_of(const SymShape &h, int64_t sid)
{
    const double b = (double)h.S0 + 0.5 * h.d;
    double r = b * b - 2.0 * h.d * (double)sid;
    r = r > 0.0 ? r : 0.0;
    int64_t g = (int64_t)((b - __builtin_sqrt(r)) / h.d);
    g = g < 0 ? 0 : (g > h.G - 1 ? h.G - 1 : g);
    while (g > 0 && h.tb(g) > sid) --g;
    while (g < h.G - 1 && h.tb(g + 1) <= sid) ++g;
    return g;
}

// 1/sqrt(v) from v_rsq_f64 with one Newton correction (relative error below
// 5e-15).
__device__ __forceinline__ double rsq_nr(double v)
{
    const double y = __builtin_amdgcn_rsq(v);
    const double e = __builtin_fma(-v, y * y, 1.0);
    return __builtin_fma(y * e, 0.5, y);
}

}  // namespace genga
