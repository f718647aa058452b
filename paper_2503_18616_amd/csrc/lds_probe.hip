// LDS bandwidth probe: the peak the step kernel's LDS roofline is set against.
//
// Every workgroup streams its own 64 KB LDS buffer with the two access forms
// the step kernel uses for particles: 16-byte reads (ds_read_b128, a
// particle's position and inverse mass) and 12-byte writes at a 16-byte
// stride (ds_write_b96, a position).  Lane l of a wave touches the 16-byte
// chunk l of a 1 KB run, so every aligned group of lanes names distinct
// banks: the probe measures the conflict-free rate.  Each workgroup records
// its shader-clock cycles (s_memtime) and its 100 MHz real-time ticks
// (s_memrealtime) between two barriers around the loop, so the host can
// state bytes per clock per CU without assuming a clock.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/xpbd_probe.h"
#include "runtime_util.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeBytes = 65536;               // per workgroup: 2 workgroups (8 waves) per CU
constexpr int kProbeUnroll = 8;                  // accesses per thread per repetition
// Repetition r reads (or writes) the half (r & 1) of the buffer, 4 KB per
// access of the workgroup: the accesses of a repetition share one per-lane
// address and differ in the instruction's immediate offset.
constexpr int kProbeHalf = kProbeBytes / 2;

// x unchanged, but opaque to the optimiser, so that the accesses of every
// repetition are issued (not merged across repetitions or hoisted)
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// kind 0: reads; each 16-byte read feeds two 64-bit adds
__global__ void __launch_bounds__(kProbeBlock) lds_read_probe(int reps, uint64_t *clocks,
                                                              uint64_t *sink)
{
    __shared__ __align__(16) ulonglong2 buf[kProbeBytes / 16];
    const int tid = threadIdx.x;
    for (int i = tid; i < kProbeBytes / 16; i += kProbeBlock)
        buf[i] = make_ulonglong2((uint64_t)i * 0x9e3779b97f4a7c15ull, (uint64_t)i + blockIdx.x);
    __syncthreads();
    const uint64_t t0 = __builtin_readcyclecounter();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    uint64_t a0 = 0, a1 = 0;
    for (int r = 0; r < reps; ++r) {
        const int base = opaque(tid + (r & 1) * (kProbeHalf / 16));
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const ulonglong2 v = buf[base + u * kProbeBlock];
            a0 += v.x;
            a1 += v.y;
        }
    }
    __syncthreads();
    const uint64_t t1 = __builtin_readcyclecounter();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    if (tid == 0) {
        clocks[2 * blockIdx.x] = t1 - t0;
        clocks[2 * blockIdx.x + 1] = r1 - r0;
    }
    if ((a0 ^ a1) == 0x5eedull)   // practically never true; keeps the loads live
        sink[0] = a0;
}

// kind 1: 12-byte writes at a 16-byte stride (a position into a float4 slot)
__global__ void __launch_bounds__(kProbeBlock) lds_write_probe(int reps, uint64_t *clocks,
                                                               uint64_t *sink)
{
    __shared__ __align__(16) float4 buf[kProbeBytes / 16];
    const int tid = threadIdx.x;
    for (int i = tid; i < kProbeBytes / 16; i += kProbeBlock)
        buf[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const uint64_t t0 = __builtin_readcyclecounter();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    float x = (float)tid, y = (float)blockIdx.x, z = 1.0f;
    for (int r = 0; r < reps; ++r) {
        const int base = opaque(tid + (r & 1) * (kProbeHalf / 16));
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            float4 &d = buf[base + u * kProbeBlock];
            d.x = x;
            d.y = y;
            d.z = z;
            x += 1.0f;
        }
    }
    __syncthreads();
    const uint64_t t1 = __builtin_readcyclecounter();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    if (tid == 0) {
        clocks[2 * blockIdx.x] = t1 - t0;
        clocks[2 * blockIdx.x + 1] = r1 - r0;
    }
    const float4 v = buf[(tid * 7) & (kProbeBytes / 16 - 1)];
    if (v.x + v.y + v.z == -1.0f)   // never true for these values; keeps the stores live
        sink[0] = 1;
}

}  // namespace

extern "C" xpbd_status xpbd_lds_probe(int32_t kind, int32_t workgroups, int32_t reps,
                                      void *hip_stream, double *out)
{
    using namespace xpbd;
    g_error.clear();
    if (!out || (kind != XPBD_PROBE_LDS_READ_B128 && kind != XPBD_PROBE_LDS_WRITE_B96))
        return fail(XPBD_E_ARG, "unknown probe kind %d or out is NULL", kind);
    if (workgroups < 1 || workgroups > (1 << 16) || reps < 1 || reps > (1 << 24))
        return fail(XPBD_E_ARG, "workgroups must be in [1, 65536], reps in [1, 2^24]");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    uint64_t *clocks = nullptr, *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    xpbd_status st = XPBD_OK;
    std::vector<uint64_t> host((size_t)workgroups * 2);
    float ms = 0.0f;
    auto run = [&]() -> hipError_t {
        hipError_t e;
        if ((e = hipMalloc(&clocks, host.size() * sizeof(uint64_t))) != hipSuccess ||
            (e = hipMalloc(&sink, sizeof(uint64_t))) != hipSuccess ||
            (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
            return e;
        auto launch = [&]() {
            if (kind == XPBD_PROBE_LDS_READ_B128)
                hipLaunchKernelGGL(lds_read_probe, dim3((unsigned)workgroups), dim3(kProbeBlock),
                                   0, s, reps, clocks, sink);
            else
                hipLaunchKernelGGL(lds_write_probe, dim3((unsigned)workgroups), dim3(kProbeBlock),
                                   0, s, reps, clocks, sink);
            return hipGetLastError();
        };
        if ((e = launch()) != hipSuccess)   // untimed first launch
            return e;
        if ((e = hipEventRecord(e0, s)) != hipSuccess || (e = launch()) != hipSuccess ||
            (e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
            return e;
        return hipMemcpy(host.data(), clocks, host.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
    };
    const hipError_t e = run();
    if (e != hipSuccess)
        st = fail(XPBD_E_HIP, "LDS probe: %s", hipGetErrorString(e));
    if (clocks)
        (void)hipFree(clocks);
    if (sink)
        (void)hipFree(sink);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (st != XPBD_OK)
        return st;
    double cycles = 0.0, ticks = 0.0;
    for (int32_t w = 0; w < workgroups; ++w) {
        cycles += (double)host[2 * (size_t)w];
        ticks += (double)host[2 * (size_t)w + 1];
    }
    const double bytes_per_access = kind == XPBD_PROBE_LDS_READ_B128 ? 16.0 : 12.0;
    out[0] = ms;
    out[1] = bytes_per_access * kProbeBlock * kProbeUnroll * (double)reps * workgroups;
    out[2] = cycles / workgroups;
    out[3] = ticks / workgroups;
    return XPBD_OK;
}
