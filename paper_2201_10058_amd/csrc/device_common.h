// Device helpers shared by the kick and its adjoint.
#pragma once

#include "genga_internal.h"

namespace genga {

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

// Changeover weight K(y), y = (r - 0.1 rho) / (0.9 rho) (Chambers 1999 eq. 10).
__device__ __forceinline__ double changeover_k(double r, double rho)
{
    const double yv = (r - 0.1 * rho) / (0.9 * rho);
    if (!(yv > 0.0)) return 0.0;
    if (yv >= 1.0) return 1.0;
    const double y2 = yv * yv;
    return y2 / (2.0 * y2 - 2.0 * yv + 1.0);
}

// K(y) of the same changeover on a precomputed y: the division by
// 2y^2 - 2y + 1 (in [1/2, 1] on the band) by v_rcp_f64 and two Newton steps.
__device__ __forceinline__ double changeover_of_y(double yv)
{
    if (!(yv > 0.0)) return 0.0;
    if (yv >= 1.0) return 1.0;
    const double y2 = yv * yv;
    const double q = __builtin_fma(2.0, y2 - yv, 1.0);
    double t = __builtin_amdgcn_rcp(q);
    t = __builtin_fma(t, __builtin_fma(-q, t, 1.0), t);
    t = __builtin_fma(t, __builtin_fma(-q, t, 1.0), t);
    return y2 * t;
}

// K(y) and dK/dy = 2y(1 - y) / q^2, q = 2y^2 - 2y + 1, with one reciprocal
// of q (v_rcp_f64 and two Newton steps); both zero below the band, K = 1 and
// dK/dy = 0 above it.
__device__ __forceinline__ void changeover_kdk_of_y(double yv, double &K, double &dK)
{
    if (!(yv > 0.0)) {
        K = 0.0;
        dK = 0.0;
        return;
    }
    if (yv >= 1.0) {
        K = 1.0;
        dK = 0.0;
        return;
    }
    const double y2 = yv * yv;
    const double q = __builtin_fma(2.0, y2 - yv, 1.0);
    double t = __builtin_amdgcn_rcp(q);
    t = __builtin_fma(t, __builtin_fma(-q, t, 1.0), t);
    t = __builtin_fma(t, __builtin_fma(-q, t, 1.0), t);
    K = y2 * t;
    dK = (2.0 * (yv - y2)) * (t * t);
}

// sum_{s < ns} p[s * stride] in slice order; the loads of 8 slices are issued
// before their additions, whose order is unchanged.
__device__ __forceinline__ double ordered_sum(const double *p, size_t stride, int ns)
{
    double acc = 0.0;
    int s = 0;
    for (; s + 8 <= ns; s += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[(size_t)(s + k) * stride];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
    }
    for (; s < ns; ++s) acc += p[(size_t)s * stride];
    return acc;
}

// max of two non-negative doubles in one v_max_f64 (the generic fmax adds
// NaN-quieting canonicalisations; the critical radii are validated instead).
__device__ __forceinline__ double vmax_f64(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ float vmax_f32(float a, float b)
{
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// binary32 mass and pre-check radius packed in the fourth double of a tile entry
__device__ __forceinline__ double pack_f32x2(float lo, float hi)
{
    return __hiloint2double(__float_as_int(hi), __float_as_int(lo));
}

// rho_ij^2 = max(rc_i^2, rc_j^2) (= fl(max(rc_i, rc_j)^2): rounding is monotone).
__device__ __forceinline__ double rho2_of(double rci, double rcj)
{
    const double a = rci * rci, b = rcj * rcj;
    return a > b ? a : b;
}

// Block-wide exclusive scan of one int64 per thread.
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

template <int NT>
__device__ int64_t block_excl_scan(int64_t v, int64_t *total, int64_t *smem /* NT/64 */)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t inc = wave_incl_scan(v);
    if (lane == 63) smem[w] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        const int64_t t = smem[k];
        if (k < w) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Largest value over the 64 lanes of a wave (all active), in every lane;
// fmax ignores a NaN operand.
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = __builtin_fmax(v, __shfl_xor(v, off));
    return v;
}

// High word of an upper bound of the largest of the 64 lanes' values (all
// lanes active, every value a non-negative double), in a scalar register:
// the largest high word over the wave.  For non-negative doubles the high
// word (as a signed int) orders the values, so bound_of_hi(h) (the low word
// set to all ones) is at least every lane's value and above their maximum by
// less than 2^-20 of it.  The maximum runs over DPP row shifts and row
// broadcasts (no address registers, unlike a butterfly of ds_bpermute); lane
// 63 ends with it.
__device__ __forceinline__ int wave_max_hi(double v)
{
    int h = __double2hiint(v);
    h = max(h, __builtin_amdgcn_update_dpp(h, h, 0x111, 0xf, 0xf, false));   // row_shr:1
    h = max(h, __builtin_amdgcn_update_dpp(h, h, 0x112, 0xf, 0xf, false));   // row_shr:2
    h = max(h, __builtin_amdgcn_update_dpp(h, h, 0x114, 0xf, 0xf, false));   // row_shr:4
    h = max(h, __builtin_amdgcn_update_dpp(h, h, 0x118, 0xf, 0xf, false));   // row_shr:8
    h = max(h, __builtin_amdgcn_update_dpp(h, h, 0x142, 0xa, 0xf, false));   // row_bcast:15
    h = max(h, __builtin_amdgcn_update_dpp(h, h, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(h, 63);
}

__device__ __forceinline__ double bound_of_hi(int h) { return __hiloint2double(h, (int)0xffffffff); }

// A value the same in every lane, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

}  // namespace genga
