// HBM copy ceiling of the current device: a streaming device-to-device copy
// (16-byte loads and stores, grid-stride, four loads in flight per thread)
// timed with HIP events over a sweep of launch shapes.  It gives the rate a
// kernel that reads and writes every byte once can reach in practice, next
// to which the plotter's memory-bound kernels are judged.  Standalone
// program: `copy_probe [GiB]` (default 8).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define CK(call)                                                                   \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));             \
            return 1;                                                              \
        }                                                                          \
    } while (0)

__global__ void copy16(const uint4 *__restrict__ a, uint4 *__restrict__ b, size_t n) {
    const size_t st = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * st < n; i += 4 * st) {
        const uint4 x0 = a[i], x1 = a[i + st], x2 = a[i + 2 * st], x3 = a[i + 3 * st];
        b[i] = x0;
        b[i + st] = x1;
        b[i + 2 * st] = x2;
        b[i + 3 * st] = x3;
    }
    for (; i < n; i += st) b[i] = a[i];
}

int main(int argc, char **argv) {
    const size_t gib = argc > 1 ? strtoull(argv[1], nullptr, 10) : 8;
    const size_t bytes = gib << 30, n = bytes / sizeof(uint4);
    uint4 *a = nullptr, *b = nullptr;
    CK(hipMalloc(&a, bytes));
    CK(hipMalloc(&b, bytes));
    CK(hipMemset(a, 1, bytes));
    CK(hipMemset(b, 2, bytes));
    CK(hipDeviceSynchronize());
    hipEvent_t s, e;
    CK(hipEventCreate(&s));
    CK(hipEventCreate(&e));
    double best = 0;
    for (int grid : {1024, 2048, 4096, 8192, 16384, 32768}) {
        for (int blk : {256, 512, 1024}) {
            hipLaunchKernelGGL(copy16, dim3(grid), dim3(blk), 0, 0, a, b, n);
            CK(hipDeviceSynchronize());
            CK(hipEventRecord(s));
            for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(copy16, dim3(grid), dim3(blk), 0, 0, a, b, n);
            CK(hipEventRecord(e));
            CK(hipEventSynchronize(e));
            float ms = 0;
            CK(hipEventElapsedTime(&ms, s, e));
            ms /= 5;
            const double tbps = 2.0 * (double)bytes / (ms * 1e-3) / 1e12;
            if (tbps > best) best = tbps;
            printf("grid %6d block %4d: %.3f ms  %.2f TB/s read+write\n", grid, blk, ms, tbps);
        }
    }
    printf("best: %.2f TB/s read+write (%zu GiB copied)\n", best, gib);
    CK(hipFree(a));
    CK(hipFree(b));
    return 0;
}
