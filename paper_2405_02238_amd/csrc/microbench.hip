// Measurement kernels behind two design choices of the library, exported
// for the benchmark harness:
//  - the modular product: FP64 (arith.h, the form every kernel uses) against
//    64-bit integer Shoup and Barrett products on gfx950's integer units;
//  - plain HBM streaming (read-only and copy), the practical ceiling the
//    memory-bound inner products are compared with.
// Nothing in the HE path calls these.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hegmm.h"
#include "arith.h"
#include "context.h"
#include "dev_common.h"

namespace hg {
namespace {

constexpr int MB_THREADS = 256;
constexpr int MB_CHAINS = 4;   // independent products per thread (latency hiding)

// Shoup: w' = floor(w 2^64 / q); a w mod q = a w - hi(a w') q, minus q at most once.
__device__ __forceinline__ uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    const uint64_t qh = __umul64hi(a, wp);
    uint64_t r = a * w - qh * q;
    return r >= q ? r - q : r;
}

// Barrett for q < 2^50: x = a b < 2^100; q1 = x >> 49; q3 = (q1 mu) >> 51 with
// mu = floor(2^100 / q); r = x - q3 q, minus q at most twice.
__device__ __forceinline__ uint64_t mul_barrett(uint64_t a, uint64_t b, uint64_t mu, uint64_t q) {
    const uint64_t lo = a * b, hi = __umul64hi(a, b);
    const uint64_t q1 = (hi << 15) | (lo >> 49);
    const uint64_t plo = q1 * mu, phi = __umul64hi(q1, mu);
    const uint64_t q3 = (phi << 13) | (plo >> 51);
    uint64_t r = lo - q3 * q;
    if (r >= q) r -= q;
    if (r >= q) r -= q;
    return r;
}

// Every thread runs MB_CHAINS independent chains x <- x * w mod q of `iters`
// products each and writes the chains' sum (so that nothing is folded away).
__global__ void __launch_bounds__(MB_THREADS)
k_mb_fp64(double *out, double q, double qi, double w, int iters) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x[MB_CHAINS];
#pragma unroll
    for (int c = 0; c < MB_CHAINS; ++c) x[c] = (double)((id * MB_CHAINS + c) % 1000003) + 1.0;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < MB_CHAINS; ++c) x[c] = mulm(x[c], w, q, qi);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < MB_CHAINS; ++c) s += x[c];
    out[id] = s;
}

__global__ void __launch_bounds__(MB_THREADS)
k_mb_shoup(uint64_t *out, uint64_t q, uint64_t w, uint64_t wp, int iters) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x[MB_CHAINS];
#pragma unroll
    for (int c = 0; c < MB_CHAINS; ++c) x[c] = (id * MB_CHAINS + c) % 1000003 + 1;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < MB_CHAINS; ++c) x[c] = mul_shoup(x[c], w, wp, q);
    uint64_t s = 0;
#pragma unroll
    for (int c = 0; c < MB_CHAINS; ++c) s += x[c];
    out[id] = s;
}

__global__ void __launch_bounds__(MB_THREADS)
k_mb_barrett(uint64_t *out, uint64_t q, uint64_t w, uint64_t mu, int iters) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x[MB_CHAINS];
#pragma unroll
    for (int c = 0; c < MB_CHAINS; ++c) x[c] = (id * MB_CHAINS + c) % 1000003 + 1;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < MB_CHAINS; ++c) x[c] = mul_barrett(x[c], w, mu, q);
    uint64_t s = 0;
#pragma unroll
    for (int c = 0; c < MB_CHAINS; ++c) s += x[c];
    out[id] = s;
}

// Streaming: each thread moves 16-byte words in a grid-stride loop.
__global__ void __launch_bounds__(MB_THREADS) k_mb_read(const uint4 *in, uint4 *out, size_t n) {
    uint32_t acc = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint4 v = in[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9e3779b9u) out[0] = make_uint4(acc, 0, 0, 0);   // keeps the loads; practically never taken
}

__global__ void __launch_bounds__(MB_THREADS) k_mb_copy(const uint4 *in, uint4 *out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

}  // namespace
}  // namespace hg

extern "C" hg_status hg_bench_modmul(int device, int form, uint64_t q, int blocks, int iters, int reps,
                                     double *out_per_s, uint64_t *checksum) {
    using namespace hg;
    if (form < 0 || form > 2 || blocks < 1 || iters < 1 || reps < 1 || !out_per_s || q <= (1ULL << 49) ||
        q >= (1ULL << 50) || !(q & 1))
        return HG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return HG_EDEVICE;
    const size_t n = (size_t)blocks * MB_THREADS;
    void *buf = nullptr;
    if (hipMalloc(&buf, n * 8) != hipSuccess) return HG_ENOMEM;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const uint64_t w = q / 3 + 12345;
    const uint64_t wp = (uint64_t)(((unsigned __int128)w << 64) / q);
    const uint64_t mu = (uint64_t)(((unsigned __int128)1 << 100) / q);
    auto run = [&] {
        if (form == 0)
            hipLaunchKernelGGL(k_mb_fp64, dim3(blocks), dim3(MB_THREADS), 0, nullptr, (double *)buf, (double)q,
                               1.0 / (double)q, (double)w, iters);
        else if (form == 1)
            hipLaunchKernelGGL(k_mb_shoup, dim3(blocks), dim3(MB_THREADS), 0, nullptr, (uint64_t *)buf, q, w, wp, iters);
        else
            hipLaunchKernelGGL(k_mb_barrett, dim3(blocks), dim3(MB_THREADS), 0, nullptr, (uint64_t *)buf, q, w, mu,
                               iters);
    };
    run();   // warm-up
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) run();
    (void)hipEventRecord(e1, nullptr);
    hipError_t err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    uint64_t sum = 0;
    if (err == hipSuccess && checksum) {
        uint64_t first[8] = {0};
        err = hipMemcpy(first, buf, sizeof(first), hipMemcpyDeviceToHost);
        for (uint64_t v : first) sum ^= v;
        *checksum = sum;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (err != hipSuccess) return HG_EDEVICE;
    *out_per_s = (double)n * MB_CHAINS * iters * reps / (ms * 1e-3);
    return HG_OK;
}

extern "C" hg_status hg_bench_stream(int device, size_t bytes, int mode, int reps, double *out_bytes_per_s) {
    using namespace hg;
    if (mode < 0 || mode > 1 || bytes < (1 << 20) || reps < 1 || !out_bytes_per_s) return HG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return HG_EDEVICE;
    const size_t n = bytes / 16;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, n * 16) != hipSuccess) return HG_ENOMEM;
    if (hipMalloc(&b, n * 16) != hipSuccess) {
        (void)hipFree(a);
        return HG_ENOMEM;
    }
    (void)hipMemset(a, 1, n * 16);
    hipDeviceProp_t prop;
    (void)hipGetDeviceProperties(&prop, device);
    const int grid = prop.multiProcessorCount * 8;
    auto run = [&] {
        if (mode == 0)
            hipLaunchKernelGGL(k_mb_read, dim3(grid), dim3(MB_THREADS), 0, nullptr, (const uint4 *)a, (uint4 *)b, n);
        else
            hipLaunchKernelGGL(k_mb_copy, dim3(grid), dim3(MB_THREADS), 0, nullptr, (const uint4 *)a, (uint4 *)b, n);
    };
    run();
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) run();
    (void)hipEventRecord(e1, nullptr);
    hipError_t err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (err != hipSuccess) return HG_EDEVICE;
    const double moved = (double)n * 16 * (mode == 0 ? 1 : 2) * reps;
    *out_bytes_per_s = moved / (ms * 1e-3);
    return HG_OK;
}
