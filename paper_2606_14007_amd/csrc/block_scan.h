// Wavefront and work-group scans for wave64 (CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vxd {

constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// Exclusive scan of one value per thread over the work-group.  s_wave needs
// BLOCK / 64 + 1 entries.  Returns the exclusive prefix; *total gets the sum.
// Every thread of the block must call it (it contains barriers).
template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T *s_wave, T *total) {
    static_assert(BLOCK % kWave == 0 && BLOCK / kWave <= kWave, "block shape");
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(x);
    if (lane == kWave - 1) s_wave[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        T w = lane < NW ? s_wave[lane] : T(0);
        T wi = wave_inclusive_scan(w);
        if (lane < NW) s_wave[lane] = wi - w;  // exclusive per-wave base
        if (lane == NW - 1) s_wave[NW] = wi;   // grand total
    }
    __syncthreads();
    T res = inc - x + s_wave[wid];
    *total = s_wave[NW];
    __syncthreads();  // s_wave may be reused right after
    return res;
}

template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T x, T *s_wave) {
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    T w = wave_sum(x);
    if (lane == 0) s_wave[wid] = w;
    __syncthreads();
    T t = T(0);
#pragma unroll
    for (int i = 0; i < NW; ++i) t += s_wave[i];
    __syncthreads();
    return t;
}

// In-place exclusive scan of s[0..n) held in LDS; n <= BLOCK * per-thread
// items.  Each thread owns a contiguous run.  Returns the total.
template <int BLOCK, typename T>
__device__ __forceinline__ T lds_exclusive_scan(T *s, int n, T *s_wave) {
    const int per = (n + BLOCK - 1) / BLOCK;
    const int lo = min((int)threadIdx.x * per, n);
    const int hi = min(lo + per, n);
    T sum = T(0);
    for (int i = lo; i < hi; ++i) sum += s[i];
    T total;
    T run = block_exclusive_scan<BLOCK>(sum, s_wave, &total);
    for (int i = lo; i < hi; ++i) {
        T c = s[i];
        s[i] = run;
        run += c;
    }
    __syncthreads();
    return total;
}

}  // namespace vxd
