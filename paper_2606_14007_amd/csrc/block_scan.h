// Wavefront and work-group scans for wave64 (CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vxd {

constexpr int kWave = 64;

// Cross-lane moves of the GFX9 data-parallel (DPP) modifier.  A row is 16
// lanes; lanes whose source lies outside the row, and lanes of rows left
// out by ROW_MASK, read zero.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, true);
}
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;  // lane 15 of each row to the whole next row
constexpr int kDppRowBcast31 = 0x143;  // lane 31 to rows 2 and 3

// One scan step: x += the value DPP control CTRL brings in (zero where it
// brings nothing).  64-bit values move as two halves and add with a carry.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_add(uint32_t &x) {
    x += dpp_u32<CTRL, ROW_MASK>(x);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_add(uint32_t &lo, uint32_t &hi) {
    const uint32_t slo = dpp_u32<CTRL, ROW_MASK>(lo), shi = dpp_u32<CTRL, ROW_MASK>(hi);
    unsigned int carry;
    lo = __builtin_addc(lo, slo, 0u, &carry);
    hi = hi + shi + carry;
}

// Inclusive scan over the first N lanes of a wave (N = 64: all of them),
// for 32- and 64-bit integers: shifts by 1, 2, 4 and 8 lanes inside each
// row of 16 (Hillis-Steele), then row 0's total added to row 1 and row 2's
// to row 3, then lane 31's (rows 0 and 1) to rows 2 and 3.  Steps that
// cannot reach inside the first N lanes are left out.  Every lane of the
// wave must be active.
template <int N = kWave, typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit integers");
    static_assert(N == 2 || N == 4 || N == 8 || N == 16 || N == kWave, "lane count");
    if constexpr (sizeof(T) == 4) {
        uint32_t v = (uint32_t)x;
        dpp_add<kDppRowShr1, 0xF>(v);
        if constexpr (N > 2) dpp_add<kDppRowShr2, 0xF>(v);
        if constexpr (N > 4) dpp_add<kDppRowShr4, 0xF>(v);
        if constexpr (N > 8) dpp_add<kDppRowShr8, 0xF>(v);
        if constexpr (N > 16) {
            dpp_add<kDppRowBcast15, 0xA>(v);
            dpp_add<kDppRowBcast31, 0xC>(v);
        }
        return (T)v;
    } else {
        uint32_t lo = (uint32_t)(uint64_t)x, hi = (uint32_t)((uint64_t)x >> 32);
        dpp_add<kDppRowShr1, 0xF>(lo, hi);
        if constexpr (N > 2) dpp_add<kDppRowShr2, 0xF>(lo, hi);
        if constexpr (N > 4) dpp_add<kDppRowShr4, 0xF>(lo, hi);
        if constexpr (N > 8) dpp_add<kDppRowShr8, 0xF>(lo, hi);
        if constexpr (N > 16) {
            dpp_add<kDppRowBcast15, 0xA>(lo, hi);
            dpp_add<kDppRowBcast31, 0xC>(lo, hi);
        }
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

// Sum over the 64 lanes of a wave (every lane active), the same in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
    x = wave_inclusive_scan(x);
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_readlane((int)x, kWave - 1);
    } else {
        const uint64_t u = (uint64_t)x;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, kWave - 1);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), kWave - 1);
        return (T)((uint64_t)lo | ((uint64_t)hi << 32));
    }
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
    T inc;
    if constexpr (sizeof(T) == 8) {
        // A wave whose values are all below 2^26 sums below 2^32: it scans
        // in 32 bits (a branch the whole wave takes the same way).
        if (__ballot((uint64_t)x >= (1ull << 26)) == 0)
            inc = (T)wave_inclusive_scan((uint32_t)(uint64_t)x);
        else
            inc = wave_inclusive_scan(x);
    } else {
        inc = wave_inclusive_scan(x);
    }
    if (lane == kWave - 1) s_wave[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        T w = lane < NW ? s_wave[lane] : T(0);
        T wi = wave_inclusive_scan<(NW <= 2 ? 2 : NW <= 4 ? 4 : NW <= 8 ? 8 : NW <= 16 ? 16 : kWave)>(w);
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
