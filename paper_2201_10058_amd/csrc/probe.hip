// Issue-rate probe: sustained throughput of the vector instructions the kick
// is built from, measured on the device the library runs on.  Each kernel
// runs independent dependency chains (8 per lane, 8 waves per SIMD), so the
// measured time is the issue cost, not the latency.
#include "genga_internal.h"

namespace genga {
namespace {

constexpr int PB = 256;    // threads per probe block
constexpr int CH = 8;      // independent chains per lane

enum ProbeOp : int {
    P_FMA64 = 0,
    P_MUL64 = 1,
    P_ADD64 = 2,
    P_RSQ64 = 3,
    P_FMA32 = 4,
    P_RSQ32 = 5,
    P_NOPS = 6
};

template <int OP>
__global__ __launch_bounds__(PB) void k_probe(double *out, int iters, double a, double b)
{
    if (OP == P_FMA32 || OP == P_RSQ32) {
        float v[CH];
        for (int k = 0; k < CH; ++k) v[k] = 1.0f + 1e-3f * (float)(threadIdx.x + k);
        const float af = (float)a, bf = (float)b;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                if (OP == P_FMA32) v[k] = __builtin_fmaf(v[k], af, bf);
                else v[k] = __builtin_amdgcn_rsqf(v[k]);
            }
        }
        float s = 0.0f;
        for (int k = 0; k < CH; ++k) s += v[k];
        out[(size_t)blockIdx.x * PB + threadIdx.x] = s;
        return;
    }
    double v[CH];
    for (int k = 0; k < CH; ++k) v[k] = 1.0 + 1e-3 * (double)(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (OP == P_FMA64) v[k] = __builtin_fma(v[k], a, b);
            else if (OP == P_MUL64) v[k] = v[k] * a;
            else if (OP == P_ADD64) v[k] = v[k] + b;
            else v[k] = __builtin_amdgcn_rsq(v[k]);
        }
    }
    double s = 0.0;
    for (int k = 0; k < CH; ++k) s += v[k];
    out[(size_t)blockIdx.x * PB + threadIdx.x] = s;
}

template <int OP>
hipError_t launch_probe(double *buf, int blocks, int iters, hipStream_t s)
{
    // a, b keep every chain finite: |a| <= 1 and b small
    hipLaunchKernelGGL(k_probe<OP>, dim3((unsigned)blocks), dim3(PB), 0, s, buf, iters,
                       OP == P_MUL64 ? 0.9999999 : 0.999999, 1e-6);
    return hipGetLastError();
}

}  // namespace
}  // namespace genga

using namespace genga;

extern "C" {

size_t genga_probe_issue_rates_bytes(void)
{
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    return sizeof(double) * (size_t)PB * (size_t)(cu * 8);
}

int genga_probe_issue_rates(double *cycles, void *buf, size_t buf_bytes, void *stream)
{
    if (!cycles || !buf) return GENGA_E_INVAL;
    int dev = 0, cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cu <= 0) {
        set_hip_error(e);
        return GENGA_E_HIP;
    }
    const int blocks = cu * 8;   // 8 blocks of 4 waves per CU: 8 waves per SIMD
    if (buf_bytes < sizeof(double) * (size_t)PB * (size_t)blocks) return GENGA_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) {
        set_hip_error(e);
        return GENGA_E_HIP;
    }
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_hip_error(e);
        return GENGA_E_HIP;
    }
    const int iters = 4096;
    int rc = GENGA_OK;
    for (int op = 0; op < P_NOPS && rc == GENGA_OK; ++op) {
        float best = -1.0f;
        for (int rep = 0; rep < 3; ++rep) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) {
                switch (op) {
                case P_FMA64: e = launch_probe<P_FMA64>((double *)buf, blocks, iters, s); break;
                case P_MUL64: e = launch_probe<P_MUL64>((double *)buf, blocks, iters, s); break;
                case P_ADD64: e = launch_probe<P_ADD64>((double *)buf, blocks, iters, s); break;
                case P_RSQ64: e = launch_probe<P_RSQ64>((double *)buf, blocks, iters, s); break;
                case P_FMA32: e = launch_probe<P_FMA32>((double *)buf, blocks, iters, s); break;
                default: e = launch_probe<P_RSQ32>((double *)buf, blocks, iters, s); break;
                }
            }
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                set_hip_error(e);
                rc = GENGA_E_HIP;
                break;
            }
            if (best < 0.0f || ms < best) best = ms;
        }
        if (rc == GENGA_OK) {
            // wave64 instructions per SIMD: blocks * 4 waves * iters * CH / (cu * 4)
            const double per_simd = (double)blocks * 4.0 * iters * CH / (4.0 * cu);
            cycles[op] = (double)best * 1e-3 * 2.4e9 / per_simd;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
