// Bench-only microbenchmark (not part of the library's C-ABI; built into libqsd_bench.so and
// loaded by bench.py --gather-ceiling): the random-gather rate that bounds hash probing.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

// Each lane issues `ilp` independent random 4-byte loads per iteration from an array of
// mask + 1 words (indices from a linear congruential generator, masked in range).
template <int ILP>
__global__ __launch_bounds__(256) void k_gather(const uint32_t *__restrict__ a, uint32_t mask, int iters,
                                                uint32_t *__restrict__ out) {
    uint32_t st[ILP];
    const uint32_t tid = blockIdx.x * 256 + threadIdx.x;
#pragma unroll
    for (int k = 0; k < ILP; ++k) st[k] = tid * 2654435761u + (uint32_t)k * 40503u + 12345u;
    uint32_t acc = 0;
    for (int it = 0; it < iters; ++it) {
        uint32_t v[ILP];
#pragma unroll
        for (int k = 0; k < ILP; ++k) {
            st[k] = st[k] * 1664525u + 1013904223u;
            v[k] = a[(st[k] >> 3) & mask];
        }
#pragma unroll
        for (int k = 0; k < ILP; ++k) {
            acc += v[k];
            st[k] ^= v[k] & 1u;
        }
    }
    out[tid] = acc;
}

}  // namespace

// Random 4-byte loads per second (`ilp` independent loads in flight per lane) from a buffer of
// `bytes` (power of two, 1 KiB .. 16 GiB) on the current device.  Returns 0, or -1 on bad
// arguments, -2 when the buffers cannot be allocated, -3 on a HIP error.
extern "C" int qsdbench_gather_rate(int64_t bytes, int32_t ilp, double *loads_per_s, void *stream) {
    if (!loads_per_s || bytes < 1024 || (bytes & (bytes - 1)) != 0 || bytes > (int64_t(1) << 34)) return -1;
    if (ilp != 1 && ilp != 2 && ilp != 4 && ilp != 8) return -1;
    hipStream_t st = (hipStream_t)stream;
    uint32_t *a = nullptr, *out = nullptr;
    const int blocks = 256 * 32;
    if (hipMalloc((void **)&a, (size_t)bytes) != hipSuccess) return -2;
    if (hipMalloc((void **)&out, (size_t)blocks * 256 * 4) != hipSuccess) {
        (void)hipFree(a);
        return -2;
    }
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -3;
    if (rc == 0) {
        const uint32_t mask = (uint32_t)(bytes / 4 - 1);
        const int iters = 64 / ilp;
        auto launch = [&]() {
            switch (ilp) {
                case 1: k_gather<1><<<blocks, 256, 0, st>>>(a, mask, iters, out); break;
                case 2: k_gather<2><<<blocks, 256, 0, st>>>(a, mask, iters, out); break;
                case 4: k_gather<4><<<blocks, 256, 0, st>>>(a, mask, iters, out); break;
                default: k_gather<8><<<blocks, 256, 0, st>>>(a, mask, iters, out); break;
            }
        };
        (void)hipMemsetAsync(a, 1, (size_t)bytes, st);
        launch();
        hipEventRecord(e0, st);
        for (int r = 0; r < 5; ++r) launch();
        hipEventRecord(e1, st);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = -3;
        else
            *loads_per_s = 5.0 * blocks * 256.0 * 64.0 / (ms * 1e-3);
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(out);
    return rc;
}
