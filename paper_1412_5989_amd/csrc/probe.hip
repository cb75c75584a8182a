// Machine ceilings for the roofline of the construction kernels, measured on
// the device they run on: the streaming-store bandwidth (the fill's output is
// a pure store stream of 8 B per entry) and the issue rate of the 64-bit XOR
// + popcount difference test (the partner scans' inner operation).
#include <hip/hip_runtime.h>

#include "ci_internal.h"

namespace ci {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Every thread stores 16-byte vectors, grid-stride over the buffer.
__global__ void __launch_bounds__(256) probe_store(u32x4* __restrict__ p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const u32x4 v = {threadIdx.x, blockIdx.x, 0u, 1u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(v, p + i);
}

// kChains independent chains of x = popcount(a ^ x) + x per lane; one step is
// one 64-bit XOR and one 64-bit popcount (the difference test of one word).
constexpr int kChains = 8;
__global__ void __launch_bounds__(256) probe_popc(uint64_t* __restrict__ out, int iters, uint64_t seed)
{
    uint64_t x[kChains];
    const uint64_t a = seed ^ ((uint64_t)threadIdx.x * 0x9e3779b97f4a7c15ull);
#pragma unroll
    for (int c = 0; c < kChains; c++) x[c] = a + (uint64_t)c * 0x632be59bd9b4e019ull;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int c = 0; c < kChains; c++) x[c] = (uint64_t)__popcll(a ^ x[c]) + (x[c] << 1);
    }
    uint64_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; c++) r ^= x[c];
    if (r == 0x1234567ull) out[threadIdx.x] = r;  // keeps the loop; practically never taken
}

}  // namespace
}  // namespace ci

namespace ci {

// Times the two probes on stream s (one warm-up launch each): returns the
// store bandwidth (bytes/s) over `bytes` of buf and the XOR + popcount steps/s.
hipError_t run_probes(void* buf, size_t bytes, hipStream_t s, double* store_bps, double* steps_per_s)
{
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    const int64_t n = (int64_t)(bytes / sizeof(u32x4));
    const unsigned sgrid = 256 * 32;
    const int reps = 5, iters = 4096;
    const unsigned pgrid = 256 * 16;
    float ms_store = 0.0f, ms_popc = 0.0f;
    hipLaunchKernelGGL(probe_store, dim3(sgrid), dim3(256), 0, s, (u32x4*)buf, n);
    e = hipEventRecord(e0, s);
    for (int k = 0; k < reps && e == hipSuccess; k++) {
        hipLaunchKernelGGL(probe_store, dim3(sgrid), dim3(256), 0, s, (u32x4*)buf, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_store, e0, e1);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(probe_popc, dim3(pgrid), dim3(256), 0, s, (uint64_t*)buf, iters, 1ull);
        e = hipEventRecord(e0, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(probe_popc, dim3(pgrid), dim3(256), 0, s, (uint64_t*)buf, iters, 7ull);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_popc, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    *store_bps = (double)reps * (double)n * sizeof(u32x4) / (ms_store * 1e-3);
    *steps_per_s = (double)pgrid * 256 * iters * kChains / (ms_popc * 1e-3);
    return hipSuccess;
}

}  // namespace ci
