// Peak-rate probes for the roofline of the fault-simulation pass, measured
// on the device the benchmark runs on: the HBM streaming rate (a copy, every
// byte read once and written once) and the int32 vector-ALU rate (independent
// chains of single-cycle integer instructions).  They are measurement tools,
// not part of the simulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace {

// Grid-stride copy, four 16-byte loads in flight per lane before the stores.
__global__ __launch_bounds__(256) void k_stream(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// Eight independent chains, each step one v_add_u32 and one v_xor_b32 written
// out so that the compiler cannot fuse or drop them: 16 int32 VALU
// instructions per step and lane.
constexpr int kValuSteps = 2048;
constexpr int kValuOpsPerStep = 16;

__global__ __launch_bounds__(256) void k_valu(uint32_t seed, uint32_t* __restrict__ out)
{
    uint32_t a[8], b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = seed + threadIdx.x + 17u * k;
        b[k] = seed ^ (blockIdx.x * 131u + k);
    }
    for (int s = 0; s < kValuSteps; ++s) {
#pragma unroll
        for (int k = 0; k < 8; ++k) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(b[k]));
#pragma unroll
        for (int k = 0; k < 8; ++k) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(b[k]) : "v"(a[k]));
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r += a[k] ^ b[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

int num_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 0;
    return cus;
}

}  // namespace

extern "C" {

// Best HBM streaming rate over `reps` copies of `bytes` bytes (each copy reads
// `bytes` and writes `bytes`): *gbs = 2 * bytes / time, in GB/s.  Allocates
// 2 * bytes of device memory for the call.  Returns 0, or -3 when the memory
// is not available, -4 on another HIP error.
int riros_peak_hbm(uint64_t bytes, int reps, double* gbs, void* stream)
{
    if (!gbs || bytes < 16 || reps < 1) return -1;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = bytes / 16;
    uint4 *src = nullptr, *dst = nullptr;
    if (hipMalloc((void**)&src, n * 16) != hipSuccess) return -3;
    if (hipMalloc((void**)&dst, n * 16) != hipSuccess) {
        (void)hipFree(src);
        return -3;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    float best = 1e30f;
    const int cus = num_cus();
    const uint32_t blocks = (uint32_t)std::max(1, cus) * 16u;
    if (hipMemsetAsync(src, 1, n * 16, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        rc = -4;
    for (int r = 0; rc == 0 && r <= reps; ++r) {
        (void)hipEventRecord(e0, s);
        hipLaunchKernelGGL(k_stream, dim3(blocks), dim3(256), 0, s, src, dst, n);
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -4;
        if (r > 0) best = std::min(best, ms);   // the first copy also loads the code object
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (rc == 0) *gbs = 2.0 * (double)(n * 16) / (best * 1e-3) / 1e9;
    return rc;
}

// Best int32 vector-ALU rate over `reps` launches: *ops_per_s = int32
// instructions executed per second, counted per lane (64 per wavefront
// instruction).  Returns 0, or -4 on a HIP error.
int riros_peak_valu(int reps, double* ops_per_s, void* stream)
{
    if (!ops_per_s || reps < 1) return -1;
    hipStream_t s = (hipStream_t)stream;
    const int cus = num_cus();
    const uint32_t blocks = (uint32_t)std::max(1, cus) * 8u;
    const size_t threads = (size_t)blocks * 256;
    uint32_t* out = nullptr;
    if (hipMalloc((void**)&out, threads * sizeof(uint32_t)) != hipSuccess) return -3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    float best = 1e30f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -4;
    for (int r = 0; rc == 0 && r <= reps; ++r) {
        (void)hipEventRecord(e0, s);
        hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(256), 0, s, 12345u + (uint32_t)r, out);
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -4;
        if (r > 0) best = std::min(best, ms);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc == 0) *ops_per_s = (double)threads * kValuSteps * kValuOpsPerStep / (best * 1e-3);
    return rc;
}

}  // extern "C"
