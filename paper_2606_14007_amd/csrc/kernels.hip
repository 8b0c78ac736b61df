// HIP kernels of the VaultX plotter hot path for gfx950 (MI355X).
//
// Stages (paper sec. III-A): hash every nonce into Table 1, file records into
// 2^24 buckets by hash prefix, sort inside buckets, then match neighbours
// below the threshold and hash each pair into Table 2.
//
// How the work maps onto CDNA4 (the paper's per-record atomic slot claim
// into fixed-size buckets and its one-thread insertion sort are replaced):
//  * hash: one nonce per lane, BLAKE3 held in VGPRs, key in SGPRs; in a plot
//    the same kernel also does the first partition pass (the ALU-bound hash
//    hides that pass's memory traffic);
//  * bucketing: up to three MSD partition passes over the leading key bits,
//    each ranking a sub-tile's records by digit in LDS and writing every
//    digit's run contiguously, so that every "group" of keys sharing the
//    leading G bits ends up together and small enough for LDS.  A plot's
//    passes claim room for each run in fixed-size regions with one global
//    atomic per (sub-tile, digit); caller keys and chunks use a histogram
//    per tile and a column scan instead;
//  * sort: one work-group per group: LDS counting sort on the next 12 bits,
//    then an exact rank inside each (tiny) sub-bin, written to the group's
//    place in Table 1; bucket offsets come from a binary search of the
//    sorted group, and each record's pair count is stored as one byte;
//  * match + Table-2 hash: fixed chunks of Table 1, a work-group scan of the
//    count bytes and a device scan give every pair its canonical slot;
//    pairs are expanded into an LDS list and hashed one pair per lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "block_scan.h"
#include "blake3_device.h"
#include "kernels.h"

namespace vxk {

using vxd::Key;

constexpr int kMaxDigits = 1 << kMaxDigitBits;
// Match kernels: work-groups of 512 threads, chunks of up to 2048 records,
// windows of 4096 Table-2 slots.
constexpr int kMatchBlock = 512;
constexpr int kMatchCap = 2048;
constexpr int kMatchSlots = 4096;

struct TileGeom {
    // mode 0: tile t covers [t * chunk, min((t + 1) * chunk, n)).
    // mode 1: tile t is part (t % q) of q equal parts of segment s = t / q,
    //         which covers [seg[s], seg_end[s]) (seg_end = seg + 1 for
    //         back-to-back segments).
    uint32_t mode;
    uint32_t q;
    uint64_t chunk;
    uint64_t n;
    const uint32_t *seg;
    const uint32_t *seg_end;
};

__device__ __forceinline__ void tile_range(const TileGeom &g, uint32_t t, uint64_t &lo,
                                           uint64_t &hi) {
    if (g.mode == 0) {
        lo = (uint64_t)t * g.chunk;
        hi = lo + g.chunk;
        if (lo > g.n) lo = g.n;
        if (hi > g.n) hi = g.n;
    } else {
        const uint32_t s = t / g.q, part = t % g.q;
        const uint64_t a = g.seg[s], b = g.seg_end[s], len = b - a;
        lo = a + len * part / g.q;
        hi = a + len * (part + 1) / g.q;
    }
}

__device__ __forceinline__ bool rec_less(uint64_t ka, uint32_t na, uint64_t kb, uint32_t nb) {
    return ka < kb || (ka == kb && na < nb);
}

// ---------------------------------------------------------------------------
// Table-1 hash (+ first-digit histogram)
// ---------------------------------------------------------------------------

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_hash_table1(Key key, uint64_t n, uint64_t chunk,
                                                       uint64_t *__restrict__ keys,
                                                       uint32_t *__restrict__ hist,
                                                       uint32_t hist_bits) {
    __shared__ uint32_t s_hist[kMaxDigits];
    const uint32_t nd = hist ? (1u << hist_bits) : 0u;
    for (uint32_t i = threadIdx.x; i < nd; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    uint64_t lo = (uint64_t)blockIdx.x * chunk;
    uint64_t hi = lo + chunk;
    if (hi > n) hi = n;
    const uint32_t shift = 64u - hist_bits;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += BLOCK) {
        // The empty asm hides that the nonce is the loop counter: otherwise
        // the optimiser strength-reduces "uniform + nonce" sums inside the
        // rounds into extra per-iteration adds (about 70 VALU per hash).
        uint32_t nonce = (uint32_t)i;
        asm volatile("" : "+v"(nonce));
        const uint64_t a = vxd::h1(key, nonce);
        keys[i] = a;
        if (hist) atomicAdd(&s_hist[a >> shift], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += BLOCK) hist[(uint64_t)blockIdx.x * nd + d] = s_hist[d];
}

// ---------------------------------------------------------------------------
// Table-1 hash of one bucket range (chunked plots): every nonce of the tile
// is hashed and the records whose key has `prefix` in its top `pbits` bits
// are kept.  Per sub-tile of BLOCK * ITEMS nonces, wave w hashes a contiguous
// run of 64 * ITEMS nonces and packs its matches into its own LDS region
// (ballot + mbcnt), the work-group claims room for the sub-tile's matches
// with one global atomic on *count, and each wave copies its run out.  The
// output is in no particular order (the sort orders records fully); records
// past `cap` are counted but not written.
// ---------------------------------------------------------------------------

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_hash_filter(Key key, uint64_t n, uint64_t chunk, uint32_t pbits,
                                                       uint32_t prefix, uint64_t *__restrict__ out_keys,
                                                       uint32_t *__restrict__ out_nonces, uint64_t cap,
                                                       unsigned long long *__restrict__ count) {
    constexpr int NW = BLOCK / 64;
    constexpr int PER_WAVE = 64 * ITEMS;
    __shared__ uint64_t s_k[BLOCK * ITEMS];
    __shared__ uint32_t s_n[BLOCK * ITEMS];
    __shared__ uint32_t s_wc[NW];
    __shared__ unsigned long long s_base;
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    for (uint64_t base = lo; base < hi; base += (uint64_t)BLOCK * ITEMS) {
        uint32_t cnt = 0;  // matches of this wave so far (same in every lane)
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t i = base + (uint64_t)w * PER_WAVE + (uint64_t)j * 64 + lane;
            uint32_t nonce = (uint32_t)i;
            asm volatile("" : "+v"(nonce));  // as in k_hash_table1
            const uint64_t a = vxd::h1(key, nonce);
            const bool m = i < hi && (pbits == 0 || (uint32_t)(a >> (64 - pbits)) == prefix);
            const uint64_t bal = __ballot(m);
            if (m) {
                const uint32_t pos = cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                s_k[w * PER_WAVE + pos] = a;
                s_n[w * PER_WAVE + pos] = (uint32_t)i;
            }
            cnt += (uint32_t)__popcll(bal);
        }
        if (lane == 0) s_wc[w] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int x = 0; x < NW; ++x) tot += s_wc[x];
            s_base = tot ? atomicAdd(count, tot) : 0ull;
        }
        __syncthreads();
        unsigned long long wb = s_base;
        for (uint32_t x = 0; x < w; ++x) wb += s_wc[x];
        for (uint32_t p = lane; p < cnt; p += 64) {
            const unsigned long long o = wb + p;
            if (o < cap) {
                out_keys[o] = s_k[w * PER_WAVE + p];
                out_nonces[o] = s_n[w * PER_WAVE + p];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Table-1 hash fused with the first partition pass.  The digit of a key
// (its top `bits` bits) picks one of 2^bits regions of R records each; a
// region fills in no particular order, which is harmless because the group
// sort orders each group fully by (key, nonce).  Per sub-tile of BLOCK *
// ITEMS nonces the work-group hashes into registers, ranks the keys by digit
// with LDS atomics, claims room in each region with one global atomic per
// digit on fill[d], lays the sub-tile out digit by digit in LDS and writes
// every digit's run contiguously.  Work-group b takes sub-tiles
// [b * per_wg, (b + 1) * per_wg).  Records past a region's capacity are not
// written and raise VXK_DEV_STATUS_REGION_OVERFLOW (fill[d] still counts
// them).
// ---------------------------------------------------------------------------

template <int BLOCK, int ITEMS, int MAXD>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MAXD <= 64 ? 6 : 1))) void k_hash_scatter(Key key, uint64_t n, uint64_t per_wg, uint32_t bits,
                                                        uint32_t R, uint64_t *__restrict__ out_keys,
                                                        uint32_t *__restrict__ out_nonces,
                                                        uint32_t *__restrict__ fill,
                                                        uint32_t *__restrict__ status) {
    constexpr int SUB = BLOCK * ITEMS;
    constexpr int PER = (MAXD + 63) / 64;  // digits per lane of the one-wave scan
    static_assert(MAXD <= BLOCK, "one thread per digit claims its region room");
    __shared__ uint64_t s_keys[SUB];
    __shared__ uint32_t s_non[SUB];
    __shared__ uint32_t s_cnt[MAXD];      // digit counts of the sub-tile
    __shared__ uint32_t s_pos[MAXD + 1];  // their exclusive prefix, and the total
    __shared__ uint32_t s_claim[MAXD];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t nd = 1u << bits, shift = 64u - bits;
    const uint64_t nsub = (n + SUB - 1) / SUB;
    const uint64_t s0 = (uint64_t)blockIdx.x * per_wg;
    const uint64_t s1 = s0 + per_wg < nsub ? s0 + per_wg : nsub;
    bool over = false;
    if (tid < nd) s_cnt[tid] = 0;
    __syncthreads();
    for (uint64_t sub = s0; sub < s1; ++sub) {
        const uint64_t base = sub * SUB;
        uint64_t k[ITEMS];
        uint32_t slot[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t i = base + (uint64_t)j * BLOCK + tid;
            // As in k_hash_table1: keep the nonce opaque to the optimiser.
            uint32_t nonce = (uint32_t)i;
            asm volatile("" : "+v"(nonce));
            k[j] = vxd::h1(key, nonce);
            if (i < n) slot[j] = atomicAdd(&s_cnt[(uint32_t)(k[j] >> shift)], 1u);
        }
        __syncthreads();
        // Claim room in the regions (thread d <-> digit d); the atomics are in
        // flight during the scan and the LDS layout.  Wave 0 scans the counts
        // on its own (no block-wide barriers).
        uint32_t claim = 0;
        if (tid < nd) {
            const uint32_t c = s_cnt[tid];
            if (c) claim = atomicAdd(&fill[tid], c);
        }
        if (tid < 64) {
            uint32_t v[PER], sum = 0;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const uint32_t d = lane * PER + q;
                v[q] = d < nd ? s_cnt[d] : 0u;
                sum += v[q];
            }
            const uint32_t inc = vxd::wave_inclusive_scan(sum);
            uint32_t run = inc - sum;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const uint32_t d = lane * PER + q;
                if (d < nd) s_pos[d] = run;
                run += v[q];
            }
            if (lane == 63) s_pos[MAXD] = inc;
        }
        __syncthreads();
        // The counts are consumed: clear them for the next sub-tile (its
        // atomics come after the next barrier).
        if (tid < nd) s_cnt[tid] = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t i = base + (uint64_t)j * BLOCK + tid;
            if (i < n) {
                const uint32_t p = s_pos[(uint32_t)(k[j] >> shift)] + slot[j];
                s_keys[p] = k[j];
                s_non[p] = (uint32_t)i;
            }
        }
        if (tid < nd) s_claim[tid] = claim;
        __syncthreads();
        // No barrier after the write-out: the next sub-tile's LDS layout waits
        // for the barrier after its hash, which every thread reaches only once
        // its reads here are done.
        const uint32_t total = s_pos[MAXD];
        for (uint32_t e = tid; e < total; e += BLOCK) {
            const uint64_t kk = s_keys[e];
            const uint32_t d = (uint32_t)(kk >> shift);
            const uint32_t r = s_claim[d] + (e - s_pos[d]);
            if (r < R) {
                const uint64_t g = (uint64_t)d * R + r;
                out_keys[g] = kk;
                out_nonces[g] = s_non[e];
            } else {
                over = true;
            }
        }
    }
    if (over) atomicOr(status, (uint32_t)VXK_DEV_STATUS_REGION_OVERFLOW);
}

// Regions of k_hash_scatter as partition segments: region d holds records
// [d * R, d * R + min(fill[d], R)) (seg_lo / seg_hi), and its records go to
// gstart[d] = the sum of the regions before it; gstart[nd] = all records.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_region_scan(const uint32_t *__restrict__ fill, uint32_t nd, uint32_t R,
                                                       uint32_t *__restrict__ seg_lo,
                                                       uint32_t *__restrict__ seg_hi,
                                                       uint32_t *__restrict__ gstart) {
    __shared__ uint32_t s[kMaxDigits];
    __shared__ uint32_t s_wave[BLOCK / 64 + 1];
    for (uint32_t d = threadIdx.x; d < nd; d += BLOCK) {
        const uint32_t c = min(fill[d], R);
        s[d] = c;
        seg_lo[d] = d * R;
        seg_hi[d] = d * R + c;
    }
    __syncthreads();
    const uint32_t total = vxd::lds_exclusive_scan<BLOCK>(s, (int)nd, s_wave);
    for (uint32_t d = threadIdx.x; d < nd; d += BLOCK) gstart[d] = s[d];
    if (threadIdx.x == 0) gstart[nd] = total;
}

// ---------------------------------------------------------------------------
// Hash of nonce slices beside the next partition pass of slices hashed
// before, in one persistent launch.
//
// The hash is bound by the vector ALUs and leaves memory nearly idle; a
// partition pass is bound by memory and LDS and leaves the ALUs nearly idle.
// A plot hashed in slices runs, in launch i, the hash (and first-digit
// filing) of slice i beside the next-digit filing of the regions of slice
// i - 1, which launch i - 1 wrote (stream order makes them visible; no item
// waits on another).  Work-groups take items of both kinds from one ticket
// counter, interleaved in proportion to their numbers, so that every CU
// holds both kinds at once.  Both kinds share one LDS layout: a sub-tile of
// SUB records is ranked by digit with LDS atomics, each digit's run claims
// room in its region with one global atomic, and the runs are written
// contiguously.  A list may hold slices of several plots (a batch).
// ---------------------------------------------------------------------------

// The digit of a key: bits [shift, shift + bits) of the 64-bit key, where
// shift >= 32 (every partition digit lies in the 24 bucket bits), so one
// bit-field extract of the high word.
__device__ __forceinline__ uint32_t key_digit(uint64_t key, uint32_t shift, uint32_t bits) {
    return __builtin_amdgcn_ubfe((uint32_t)(key >> 32), shift - 32u, bits);
}

// Files a sub-tile of m <= BLOCK * ITEMS records, held lane-strided in k[] /
// nv[] (item j of thread t is record j * BLOCK + t), by their digit
// key_digit(key, shift, bits), shift >= 32: ranks them with LDS atomics on
// cnt[], claims room for each digit's run in region region0 + d (capacity
// R) with one global atomic on fill[], lays the sub-tile out digit by digit
// in LDS and writes every run contiguously.  A run that does not fit its
// region is cut at the region's end and the digit's claiming thread sets
// the overflow status bit.  Every output record index is below 2^32 (the
// output regions hold fewer records).  cnt[] must be zero on entry and is
// zero again on return; dst[d] receives {the output index of the record at
// LDS position 0 of digit d's run, wrapped to 32 bits; the end of the run's
// records that fit}.  before_barrier() runs between the ranking and the
// first barrier.  No barrier follows the write-out: a caller's next LDS
// layout must come after a barrier that every thread reaches only once its
// reads here are done.  Full sub-tiles (m == BLOCK * ITEMS, nearly all)
// take straight-line code without per-record bounds checks.
template <int BLOCK, int ITEMS, int MAXD, typename F>
__device__ __forceinline__ void file_records(const uint64_t (&k)[ITEMS], const uint32_t (&nv)[ITEMS], uint32_t m,
                                             uint32_t shift, uint32_t bits, uint32_t *fill, uint32_t region0,
                                             uint32_t R, uint64_t *okeys, uint32_t *ononces, uint32_t *status,
                                             uint64_t *s_keys, uint32_t *s_non, uint32_t *s_cnt, uint32_t *s_pos,
                                             uint2 *s_dst, F before_barrier) {
    constexpr int PER = (MAXD + 63) / 64;  // digits per lane of the one-wave scan
    constexpr uint32_t SUB = BLOCK * ITEMS;
    static_assert(MAXD <= BLOCK, "one thread per digit claims its region room");
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const bool full = m == SUB;
    // The digit width in a vector register, once: a vector instruction
    // takes one scalar operand here, and the extract's offset is that one.
    uint32_t vbits = bits;
    asm volatile("" : "+v"(vbits));
    uint32_t slot[ITEMS];
    if (full) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) slot[j] = atomicAdd(&s_cnt[key_digit(k[j], shift, vbits)], 1u);
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
            slot[j] = j * BLOCK + tid < m ? atomicAdd(&s_cnt[key_digit(k[j], shift, vbits)], 1u) : 0u;
    }
    before_barrier();
    __syncthreads();
    // Claim room in the regions (thread d <-> digit d); the atomics are in
    // flight during the scan and the LDS layout.  Wave 0 scans the counts.
    const uint32_t nd = 1u << bits;
    uint32_t claim = 0, c = 0;
    if (tid < nd) {
        c = s_cnt[tid];
        if (c) claim = atomicAdd(&fill[region0 + tid], c);
    }
    if (tid < 64) {
        uint32_t v[PER], sum = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t d = lane * PER + q;
            v[q] = d < nd ? s_cnt[d] : 0u;
            sum += v[q];
        }
        const uint32_t inc = vxd::wave_inclusive_scan(sum);
        uint32_t run = inc - sum;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t d = lane * PER + q;
            if (d < nd) s_pos[d] = run;
            run += v[q];
        }
    }
    __syncthreads();
    // The counts are consumed: clear them for the next sub-tile (its atomics
    // come after the next barrier).  Digit d's run starts at output index
    // (region0 + d) * R + claim and keeps the records that fit below R.
    if (tid < nd) {
        s_cnt[tid] = 0;
        const uint32_t pos = s_pos[tid];
        const uint32_t fit = claim < R ? min(c, R - claim) : 0u;
        if (fit < c) atomicOr(status, (uint32_t)VXK_DEV_STATUS_REGION_OVERFLOW);
        s_dst[tid] = make_uint2((region0 + tid) * R + claim - pos, pos + fit);
    }
    if (full) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t p = s_pos[key_digit(k[j], shift, vbits)] + slot[j];
            s_keys[p] = k[j];
            s_non[p] = nv[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
            if (j * BLOCK + tid < m) {
                const uint32_t p = s_pos[key_digit(k[j], shift, vbits)] + slot[j];
                s_keys[p] = k[j];
                s_non[p] = nv[j];
            }
    }
    __syncthreads();
    auto put = [&](uint32_t e) {
        const uint64_t kk = s_keys[e];
        const uint64_t dd = reinterpret_cast<const uint64_t *>(s_dst)[key_digit(kk, shift, vbits)];  // one read
        if (e < (uint32_t)(dd >> 32)) {
            const uint32_t g = (uint32_t)dd + e;
            okeys[g] = kk;
            ononces[g] = s_non[e];
        }
    };
    if (full) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) put(j * BLOCK + tid);
    } else {
        for (uint32_t e = tid; e < m; e += BLOCK) put(e);
    }
}

// Sub-tile x of a hash slice: hashes its nonces into k[] / nv[]; returns
// the number of records (the last sub-tile may be short).
template <int BLOCK, int ITEMS>
__device__ __forceinline__ uint32_t hash_subtile(const HashSliceDesc &H, uint32_t x, uint64_t (&k)[ITEMS],
                                                 uint32_t (&nv)[ITEMS]) {
    constexpr uint32_t SUB = BLOCK * ITEMS;
    Key key;
#pragma unroll
    for (int w = 0; w < 8; ++w) key.w[w] = H.key[w];
    const uint64_t base = (uint64_t)x * SUB;
    const uint32_t m = (uint32_t)(H.n - base < SUB ? H.n - base : SUB);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        // As in k_hash_table1: keep the nonce opaque to the optimiser.
        uint32_t nonce = (uint32_t)(H.nonce0 + base) + (uint32_t)(j * BLOCK) + threadIdx.x;
        asm volatile("" : "+v"(nonce));
        k[j] = vxd::h1(key, nonce);
        nv[j] = nonce;
    }
    return m;
}

// Sub-tile x of a pass over a slice's regions: loads region x / per's
// records [(x % per) * SUB, ...) (clamped, unconditional loads: a wave
// issues all before waiting); returns the number of records, and the
// region in *r.
template <int BLOCK, int ITEMS>
__device__ __forceinline__ uint32_t load_subtile(const PassSliceDesc &P, uint32_t x, uint64_t (&k)[ITEMS],
                                                 uint32_t (&nv)[ITEMS], uint32_t *r_out) {
    constexpr uint32_t SUB = BLOCK * ITEMS;
    const uint32_t r = x / P.per, lo = (x % P.per) * SUB;
    const uint32_t f = min(P.fill[r], P.R_in);
    const uint32_t m = lo < f ? min(SUB, f - lo) : 0u;
    *r_out = r;
    if (m) {
        const uint64_t src = (uint64_t)r * P.R_in + lo;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = j * BLOCK + threadIdx.x;
            const uint64_t ic = src + (e < m ? e : m - 1);
            k[j] = P.keys[ic];
            nv[j] = P.nonces[ic];
        }
    }
    return m;
}

// Position t of a launch's ticket order belongs to the first list while
// floor(t * frac / 2^32) grows across it (frac = ceil(n1 * 2^32 / n));
// returns whether it does, with the item index in the chosen list.
__device__ __forceinline__ bool take_first(uint64_t t, uint64_t frac, uint64_t &idx) {
    const uint64_t a0 = (t * frac) >> 32, a1 = ((t + 1) * frac) >> 32;
    idx = a1 > a0 ? a0 : t - a0;
    return a1 > a0;
}

template <int BLOCK, int ITEMS, int MAXD>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MAXD <= 128 ? 6 : 1))) void k_hash_pass(HashPassList L,
                                                                                     uint32_t *__restrict__ ticket) {
    constexpr uint32_t SUB = BLOCK * ITEMS;
    __shared__ uint64_t s_keys[SUB];
    __shared__ uint32_t s_non[SUB];
    __shared__ uint32_t s_cnt[MAXD];      // digit counts of the sub-tile
    __shared__ uint32_t s_pos[MAXD + 1];  // their exclusive prefix
    __shared__ uint2 s_dst[MAXD];
    __shared__ uint32_t s_tk[2];  // alternate, so a slow reader never sees the next ticket
    const uint32_t tid = threadIdx.x;
    const uint64_t NT = (uint64_t)L.h_items + L.p_items;
    if (tid < MAXD) s_cnt[tid] = 0;
    if (tid == 0) s_tk[0] = atomicAdd(ticket, 1u);
    __syncthreads();
    // Filing and pass loads issue at a raised wave priority, so that the
    // memory-bound phases get their few instructions out ahead of the hash
    // waves sharing the SIMD.
    __builtin_amdgcn_s_setprio(2);
    for (uint32_t it = 0;; ++it) {
        const uint64_t t = s_tk[it & 1];
        if (t >= NT) break;
        uint64_t idx;
        const bool hrole = take_first(t, L.h_frac, idx);
        uint64_t k[ITEMS];
        uint32_t nv[ITEMS];
        uint32_t m, shift, bits, R, region0;
        uint32_t *fill, *ononces, *status;
        uint64_t *okeys;
        if (hrole) {
            uint32_t x = (uint32_t)idx, s = 0;
            while (s + 1 < L.nh && x >= L.h[s].items) x -= L.h[s].items, ++s;
            const HashSliceDesc &H = L.h[s];
            __builtin_amdgcn_s_setprio(0);  // the hash: vector work that any wave's idle cycles can take
            m = hash_subtile<BLOCK, ITEMS>(H, x, k, nv);
            __builtin_amdgcn_s_setprio(2);
            shift = 64u - H.bits;
            bits = H.bits;
            R = H.R;
            region0 = 0;
            fill = H.fill;
            okeys = H.keys;
            ononces = H.nonces;
            status = H.status;
        } else {
            uint32_t x = (uint32_t)idx, s = 0;
            while (s + 1 < L.np && x >= L.p[s].items) x -= L.p[s].items, ++s;
            const PassSliceDesc &P = L.p[s];
            uint32_t r;
            m = load_subtile<BLOCK, ITEMS>(P, x, k, nv, &r);
            shift = P.shift;
            bits = P.bits;
            R = P.R_out;
            region0 = (P.r0 + r) << P.bits;
            fill = P.out_fill;
            okeys = P.out_keys;
            ononces = P.out_nonces;
            status = P.status;
        }
        // The next ticket is fetched before the first barrier and read after
        // the last one.
        file_records<BLOCK, ITEMS, MAXD>(k, nv, m, shift, bits, fill, region0, R, okeys, ononces, status, s_keys,
                                         s_non, s_cnt, s_pos, s_dst, [&]() {
                                             if (tid == 0) s_tk[(it + 1) & 1] = atomicAdd(ticket, 1u);
                                         });
    }
}

// Group starts over regions that every slice of a sliced hash holds on its
// own (the first digit's, or the first two digits' when the hash launches
// also file the third pass): gstart[d] = records of digits below d over all
// slices, each slice's region d holding min(fill[s * stride + d], R);
// gstart[nd] = all.  Any nd: blocks of kMaxDigits digits carry their sum.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_region_scan_slices(const uint32_t *__restrict__ fill, uint32_t slices,
                                                              uint32_t stride, uint32_t nd, uint32_t R,
                                                              uint32_t *__restrict__ gstart) {
    __shared__ uint32_t s[kMaxDigits];
    __shared__ uint32_t s_wave[BLOCK / 64 + 1];
    uint32_t carry = 0;  // records of the digits before this block of kMaxDigits
    for (uint32_t d0 = 0; d0 < nd; d0 += kMaxDigits) {
        const uint32_t m = min(nd - d0, (uint32_t)kMaxDigits);
        for (uint32_t d = threadIdx.x; d < m; d += BLOCK) {
            uint32_t c = 0;
            for (uint32_t q = 0; q < slices; ++q) c += min(fill[q * stride + d0 + d], R);
            s[d] = c;
        }
        __syncthreads();
        const uint32_t total = vxd::lds_exclusive_scan<BLOCK>(s, (int)m, s_wave);
        for (uint32_t d = threadIdx.x; d < m; d += BLOCK) gstart[d0 + d] = carry + s[d];
        carry += total;
        __syncthreads();  // s is refilled for the next block of digits
    }
    if (threadIdx.x == 0) gstart[nd] = carry;
}

// ---------------------------------------------------------------------------
// Digit histogram per tile
// ---------------------------------------------------------------------------

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_digit_hist(const uint64_t *__restrict__ keys,
                                                      TileGeom geom, uint32_t shift,
                                                      uint32_t bits, uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_hist[kMaxDigits];
    const uint32_t nd = 1u << bits, mask = nd - 1u;
    for (uint32_t i = threadIdx.x; i < nd; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    uint64_t lo, hi;
    tile_range(geom, blockIdx.x, lo, hi);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += BLOCK)
        atomicAdd(&s_hist[(uint32_t)(keys[i] >> shift) & mask], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += BLOCK) hist[(uint64_t)blockIdx.x * nd + d] = s_hist[d];
}

// ---------------------------------------------------------------------------
// Segmented column scan of per-tile digit histograms.
// hist/off are [rows][ncol]; segment s (one work-group) owns rows
// [s * rps, (s + 1) * rps) and starts at record seg_base[s] (0 if NULL).
// off[r][c] = seg_base + sum_{c' < c} total(s, c') + sum_{rows r' < r of s} hist[r'][c]
// gstart[s * ncol + c] = seg_base + sum_{c' < c} total(s, c'); the last
// work-group also writes gstart[n_groups], the end of the last segment
// (seg_base[nseg], or n_total without segments), so a launch over a range of
// segments leaves a complete group-start array for that range.
// ---------------------------------------------------------------------------

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_colscan(const uint32_t *__restrict__ hist,
                                                   uint32_t *__restrict__ off, uint32_t rps,
                                                   uint32_t ncol,
                                                   const uint32_t *__restrict__ seg_base,
                                                   uint32_t *__restrict__ gstart,
                                                   uint32_t n_groups, uint32_t n_total) {
    __shared__ uint32_t s_part[BLOCK];
    __shared__ uint32_t s_col[kMaxDigits];
    __shared__ uint32_t s_wave[BLOCK / 64 + 1];
    const uint32_t s = blockIdx.x;
    const uint32_t base = seg_base ? seg_base[s] : 0u;
    const uint64_t r0 = (uint64_t)s * rps;
    const uint32_t tid = threadIdx.x;
    if (ncol < BLOCK) {
        // R row slices per column, one column per thread.
        const uint32_t R = BLOCK / ncol;
        const uint32_t c = tid % ncol, q = tid / ncol;
        const uint32_t a = (uint32_t)((uint64_t)rps * q / R), b = (uint32_t)((uint64_t)rps * (q + 1) / R);
        uint32_t sum = 0;
#pragma unroll 8
        for (uint32_t r = a; r < b; ++r) sum += hist[(r0 + r) * ncol + c];
        s_part[tid] = sum;
        __syncthreads();
        if (tid < ncol) {
            uint32_t run = 0;
            for (uint32_t qq = 0; qq < R; ++qq) {
                const uint32_t v = s_part[qq * ncol + tid];
                s_part[qq * ncol + tid] = run;
                run += v;
            }
            s_col[tid] = run;
        }
        __syncthreads();
        vxd::lds_exclusive_scan<BLOCK>(s_col, (int)ncol, s_wave);
        for (uint32_t cc = tid; cc < ncol; cc += BLOCK) gstart[(uint64_t)s * ncol + cc] = base + s_col[cc];
        uint32_t run = base + s_col[c] + s_part[tid];
#pragma unroll 8
        for (uint32_t r = a; r < b; ++r) {
            const uint64_t ix = (r0 + r) * ncol + c;
            const uint32_t v = hist[ix];
            off[ix] = run;
            run += v;
        }
    } else {
        // ncol >= BLOCK: several columns per thread, every row.
        for (uint32_t c = tid; c < ncol; c += BLOCK) {
            uint32_t sum = 0;
            for (uint32_t r = 0; r < rps; ++r) sum += hist[(r0 + r) * ncol + c];
            s_col[c] = sum;
        }
        __syncthreads();
        vxd::lds_exclusive_scan<BLOCK>(s_col, (int)ncol, s_wave);
        for (uint32_t c = tid; c < ncol; c += BLOCK) {
            gstart[(uint64_t)s * ncol + c] = base + s_col[c];
            uint32_t run = base + s_col[c];
            for (uint32_t r = 0; r < rps; ++r) {
                const uint64_t ix = (r0 + r) * ncol + c;
                const uint32_t v = hist[ix];
                off[ix] = run;
                run += v;
            }
        }
    }
    if (s == gridDim.x - 1 && tid == 0) gstart[n_groups] = seg_base ? seg_base[gridDim.x] : n_total;
}

// ---------------------------------------------------------------------------
// Partition scatter: each tile streams its records in sub-tiles of
// BLOCK * ITEMS, ranks them by digit in LDS and writes every digit's run
// contiguously at the tile's running cursor for that digit.  A sub-tile's
// loads are all issued before the first is waited for.
//
// CLAIM: instead of cursors from a histogram scan, every sub-tile claims
// room for its digit runs with one global atomic per digit in fixed-size
// regions: region (s, d) of segment s and digit d holds records
// [(s * 2^bits + d) * claim.R, + claim.R) of the output, and claim.fill
// counts its records (the same scheme as k_hash_scatter, records past a
// region's capacity raise VXK_DEV_STATUS_REGION_OVERFLOW).
// ---------------------------------------------------------------------------

struct Claim {
    uint32_t *fill;
    uint32_t R;
    uint32_t *status;
};

// Where a group sort reads group g: keys / nonces from records
// [lo[g], hi[g]) of the input regions, or (keys == NULL) in place at the
// group's own start.

// Records of group g and where its Table-1 slice ends.  In place, the group
// is [gstart[g], gstart[g + 1]).  Gathered from a region, it holds that
// region's (clamped) fill: without overflow this equals the difference of
// the group starts; after a region overflowed, the difference of the last
// group of a segment also counts the records the segment lost, so the group
// takes only its own region's records and leaves the rest of its slice as a
// hole (see zero_holes).  Either way every read stays inside the group's
// region and every write below gstart[g + 1] <= the table size.
__device__ __forceinline__ uint32_t group_records(const GroupIn &in, const uint32_t *gstart, uint32_t g,
                                                  uint32_t lo) {
    const uint32_t n = gstart[g + 1] - lo;
    return in.keys ? min(n, in.hi[g] - in.lo[g]) : n;
}

// After a region overflow (VXK_DEV_STATUS_REGION_OVERFLOW) Table 1 is
// incomplete: the hole of group g, [lo + n, gstart[g + 1]), and, after the
// last group, the records past the placed total up to n_total are never
// written.  Their pair-count bytes are zeroed so that the match never takes
// partners from them (a count byte only reaches records of its own group).
__device__ __forceinline__ void zero_holes(uint8_t *pcnt, const uint32_t *gstart, uint32_t g, uint32_t G,
                                           uint32_t lo, uint32_t n, uint32_t n_total) {
    if (!pcnt) return;
    const uint32_t end = gstart[g + 1];
    for (uint32_t i = lo + n + threadIdx.x; i < end; i += blockDim.x) pcnt[i] = 0;
    if (g == (1u << G) - 1)
        for (uint32_t i = end + threadIdx.x; i < n_total; i += blockDim.x) pcnt[i] = 0;
}

template <int BLOCK, int ITEMS, int MAXD, bool CLAIM>
__global__ __launch_bounds__(BLOCK) void k_scatter(const uint64_t *__restrict__ in_keys,
                                                   const uint32_t *__restrict__ in_nonces,
                                                   uint64_t *__restrict__ out_keys,
                                                   uint32_t *__restrict__ out_nonces,
                                                   const uint32_t *__restrict__ off, TileGeom geom,
                                                   uint32_t shift, uint32_t bits, Claim claim) {
    constexpr int SUB = BLOCK * ITEMS;
    static_assert(!CLAIM || MAXD <= BLOCK, "one thread per digit claims its region room");
    __shared__ uint64_t s_keys[SUB];
    __shared__ uint32_t s_nonces[SUB];
    __shared__ uint32_t s_cursor[MAXD];
    __shared__ uint32_t s_start[MAXD + 1];
    __shared__ uint32_t s_wave[BLOCK / 64 + 1];
    const uint32_t nd = 1u << bits, mask = nd - 1u;
    const uint32_t tid = threadIdx.x;
    if (!CLAIM)
        for (uint32_t d = tid; d < nd; d += BLOCK) s_cursor[d] = off[(uint64_t)blockIdx.x * nd + d];
    // Claim mode: this tile's segment and the first of its regions.
    const uint64_t region0 = CLAIM ? (uint64_t)(blockIdx.x / geom.q) * nd : 0;
    bool over = false;
    uint64_t lo, hi;
    tile_range(geom, blockIdx.x, lo, hi);
    // Loads of a sub-tile: indices past the tile are clamped to its last
    // record (and ignored later), so every load is unconditional and a wave
    // issues all of them before it waits for any.
    auto load = [&](uint64_t b, uint64_t(&kk)[ITEMS], uint32_t(&nv)[ITEMS]) {
        if (in_nonces) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint64_t idx = b + (uint64_t)j * BLOCK + tid;
                const uint64_t ic = idx < hi ? idx : hi - 1;
                kk[j] = in_keys[ic];
                nv[j] = in_nonces[ic];
            }
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint64_t idx = b + (uint64_t)j * BLOCK + tid;
                kk[j] = in_keys[idx < hi ? idx : hi - 1];
                nv[j] = (uint32_t)idx;
            }
        }
    };
    // The histogram-based scatter (a lone 8192-record work-group per CU)
    // loads the next sub-tile into registers before the current one's LDS
    // work and stores.  The claiming scatter does not: there the prefetch
    // measured neutral, and its registers went into larger sub-tiles.
    constexpr bool PREFETCH = !CLAIM;
    uint64_t nk[ITEMS];
    uint32_t nn[ITEMS];
    if (PREFETCH && lo < hi) load(lo, nk, nn);
    for (uint64_t base = lo; base < hi; base += SUB) {
        uint64_t k[ITEMS];
        uint32_t n[ITEMS], slot[ITEMS];
        if (PREFETCH) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                k[j] = nk[j];
                n[j] = nn[j];
            }
        } else {
            load(base, k, n);
        }
        for (uint32_t d = tid; d < nd; d += BLOCK) s_start[d] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t idx = base + (uint64_t)j * BLOCK + tid;
            if (idx < hi) slot[j] = atomicAdd(&s_start[(uint32_t)(k[j] >> shift) & mask], 1u);
        }
        if (PREFETCH) {
            const uint64_t nbase = base + SUB;
            if (nbase < hi) load(nbase, nk, nn);
        }
        __syncthreads();
        // Claim mode: thread d claims digit d's room; the atomic is in
        // flight during the scan and the LDS layout.
        uint32_t got = 0;
        if (CLAIM && tid < nd) {
            const uint32_t c = s_start[tid];
            if (c) got = atomicAdd(&claim.fill[region0 + tid], c);
        }
        const uint32_t total = vxd::lds_exclusive_scan<BLOCK>(s_start, (int)nd, s_wave);
        if (tid == 0) s_start[nd] = total;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t idx = base + (uint64_t)j * BLOCK + tid;
            if (idx < hi) {
                const uint32_t p = s_start[(uint32_t)(k[j] >> shift) & mask] + slot[j];
                s_keys[p] = k[j];
                s_nonces[p] = n[j];
            }
        }
        if (CLAIM && tid < nd) s_cursor[tid] = got;
        __syncthreads();
        for (uint32_t e = tid; e < total; e += BLOCK) {
            const uint64_t kk = s_keys[e];
            const uint32_t d = (uint32_t)(kk >> shift) & mask;
            if (CLAIM) {
                const uint32_t r = s_cursor[d] + (e - s_start[d]);
                if (r < claim.R) {
                    const uint64_t g = (region0 + d) * claim.R + r;
                    out_keys[g] = kk;
                    out_nonces[g] = s_nonces[e];
                } else {
                    over = true;
                }
            } else {
                const uint64_t g = (uint64_t)s_cursor[d] + (e - s_start[d]);
                out_keys[g] = kk;
                out_nonces[g] = s_nonces[e];
            }
        }
        __syncthreads();
        if (!CLAIM)
            for (uint32_t d = tid; d < nd; d += BLOCK) s_cursor[d] += s_start[d + 1] - s_start[d];
        __syncthreads();
    }
    if (CLAIM && over) atomicOr(claim.status, (uint32_t)VXK_DEV_STATUS_REGION_OVERFLOW);
}

// Claimed regions as segments of the next pass: counts clamped to the
// capacity R (in place), region r covering [r * R, r * R + count).
__global__ void k_region_bounds(uint32_t *__restrict__ fill, uint32_t r0, uint32_t nregions, uint32_t R,
                                uint32_t *__restrict__ seg_lo, uint32_t *__restrict__ seg_hi) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nregions; r += gridDim.x * blockDim.x) {
        const uint32_t c = min(fill[r], R);
        fill[r] = c;
        seg_lo[r] = (r0 + r) * R;
        seg_hi[r] = (r0 + r) * R + c;
    }
}

// ---------------------------------------------------------------------------
// Group sort in LDS (into Table 1: in place, or gathered from the last
// pass's regions), bucket offsets of the group, and (optionally) each
// record's Table-2 pair count.
// ---------------------------------------------------------------------------

constexpr int kSubBinBits = 12;
constexpr int kSubBins = 1 << kSubBinBits;

// Per-record pair counts are kept as bytes; this value means "this many or
// more" and sends the match back to the keys for that record.
constexpr uint32_t kPairCountEscape = 255;

// Pairs owned by record e of a sorted run keys[0..n): later records of the
// same bucket whose key is less than T above keys[e].  The run must end at a
// bucket boundary (a group always does).
__device__ __forceinline__ uint32_t pairs_after(const uint64_t *keys, uint32_t e, uint32_t n,
                                                uint64_t T) {
    const uint64_t ki = keys[e];
    const uint32_t bi = (uint32_t)(ki >> 40);
    uint32_t c = 0;
    for (uint32_t j = e + 1; j < n; ++j) {
        const uint64_t kj = keys[j];
        if ((uint32_t)(kj >> 40) != bi || kj - ki >= T) break;
        ++c;
    }
    return c;
}

// Table-2 pairs owned by records [e_lo, e_hi) of a sorted run keys[0, n)
// that ends at a bucket boundary, counted with a two-pointer walk (the last
// partner of a record never precedes the previous record's last partner).
// pc (may be NULL) receives each record's count as one byte, with
// kPairCountEscape standing for "that many or more".  csum (may be NULL)
// receives the counts summed per match chunk of Table 1 (chunk c = records
// [c << cb, (c + 1) << cb)), the run starting at Table-1 index `at`.
__device__ __forceinline__ uint64_t pairs_in_range(const uint64_t *keys, uint32_t e_lo, uint32_t e_hi,
                                                   uint32_t n, uint64_t T, uint8_t *pc,
                                                   unsigned long long *csum = nullptr, uint32_t cb = 0,
                                                   uint32_t at = 0) {
    uint64_t total = 0, part = 0;
    uint32_t reach = e_lo, chunk = (at + e_lo) >> cb;
    for (uint32_t e = e_lo; e < e_hi; ++e) {
        const uint64_t ki = keys[e];
        const uint32_t bi = (uint32_t)(ki >> 40);
        if (reach < e) reach = e;
        while (reach + 1 < n) {
            const uint64_t kj = keys[reach + 1];
            if ((uint32_t)(kj >> 40) != bi || kj - ki >= T) break;
            ++reach;
        }
        total += reach - e;
        if (pc) pc[e] = (uint8_t)min(reach - e, kPairCountEscape);
        if (csum) {
            if ((at + e) >> cb != chunk) {
                if (part) atomicAdd(&csum[chunk], (unsigned long long)part);
                chunk = (at + e) >> cb;
                part = 0;
            }
            part += reach - e;
        }
    }
    if (csum && part) atomicAdd(&csum[chunk], (unsigned long long)part);
    return total;
}

// Sorts the n <= CAPMAX records of a group, loaded lane-strided into k[] /
// nn[] (item j of thread t is record j * BLOCK + t), into s_keys / s_nonces
// by (key, nonce): a counting sort on the kSubBinBits key bits below the
// group prefix (sb_shift), with two 16-bit counters per LDS word in s_start
// (kSubBins / 2 + 1 words), then an exact rank inside each (tiny) sub-bin.
// A record alone in its sub-bin is in its final place after the counting
// sort; only the records that share a sub-bin are ranked and moved again.
// Every thread of the work-group calls it; it ends with a barrier, after
// which s_keys[n .. n + 3] hold all-ones sentinels and s_start holds each
// sub-bin's first position (sub-bin 2w in the low half of word w, 2w + 1
// in the high half) until the caller reuses it.
template <int BLOCK, int CAPMAX>
__device__ __forceinline__ void lds_sort_group(const uint64_t (&k)[CAPMAX / BLOCK], const uint32_t (&nn)[CAPMAX / BLOCK],
                                               uint32_t n, uint32_t sb_shift, uint64_t *s_keys,
                                               uint32_t *s_nonces, uint32_t *s_start, uint32_t *s_wave32) {
    constexpr int ITEMS = CAPMAX / BLOCK;
    constexpr int NW2 = kSubBins / 2;
    constexpr uint32_t kPlaced = 0xFFFFFFFFu;  // slot[] value of a record already in its final place
    const uint32_t tid = threadIdx.x;
    uint32_t slot[ITEMS];
    for (uint32_t i = tid; i < NW2; i += BLOCK) s_start[i] = 0;
    if (tid == 0) s_start[NW2] = n;  // start of the sub-bin past the last
    if (tid < 4) s_keys[n + tid] = ~0ull;  // sentinels after the sorted records (s_keys holds n + 4)
    __syncthreads();
    if (n == 0) return;  // uniform; k[] holds nothing
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = j * BLOCK + tid;
        if (e < n) {
            const uint32_t sb = (uint32_t)(k[j] >> sb_shift) & (kSubBins - 1);
            const uint32_t sh = (sb & 1u) << 4;
            slot[j] = (atomicAdd(&s_start[sb >> 1], 1u << sh) >> sh) & 0xFFFFu;
        }
    }
    __syncthreads();
    {
        constexpr int PERW = NW2 / BLOCK;
        uint32_t w[PERW], sum = 0;
#pragma unroll
        for (int i = 0; i < PERW; ++i) {
            w[i] = s_start[tid * PERW + i];
            sum += (w[i] & 0xFFFFu) + (w[i] >> 16);
        }
        uint32_t total;
        uint32_t run = vxd::block_exclusive_scan<BLOCK>(sum, s_wave32, &total);
#pragma unroll
        for (int i = 0; i < PERW; ++i) {
            const uint32_t lo16 = w[i] & 0xFFFFu;
            s_start[tid * PERW + i] = run | ((run + lo16) << 16);
            run += lo16 + (w[i] >> 16);
        }
    }
    __syncthreads();
    // Scatter by sub-bin.  slot[] becomes the sub-bin's start and size
    // (start | size << 16) for a record that shares it, else kPlaced.
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = j * BLOCK + tid;
        const uint32_t sb = (uint32_t)(k[j] >> sb_shift) & (kSubBins - 1);
        const uint32_t sb1 = sb + 1;
        const uint32_t b0 = (s_start[sb >> 1] >> ((sb & 1u) << 4)) & 0xFFFFu;
        const uint32_t b1 = (s_start[sb1 >> 1] >> ((sb1 & 1u) << 4)) & 0xFFFFu;
        if (e < n) {
            const uint32_t q = b0 + slot[j];
            s_keys[q] = k[j];
            s_nonces[q] = nn[j];
        }
        slot[j] = (e < n && b1 - b0 > 1u) ? (b0 | ((b1 - b0) << 16)) : kPlaced;
    }
    __syncthreads();
    // Exact rank inside a shared sub-bin; slot[] becomes the final position.
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (slot[j] != kPlaced) {
            const uint32_t b0 = slot[j] & 0xFFFFu, b1 = b0 + (slot[j] >> 16);
            uint32_t r = 0;
            for (uint32_t x = b0; x < b1; ++x) r += rec_less(s_keys[x], s_nonces[x], k[j], nn[j]);
            slot[j] = b0 + r;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (slot[j] != kPlaced) {
            s_keys[slot[j]] = k[j];
            s_nonces[slot[j]] = nn[j];
        }
    }
    __syncthreads();
}


// LDS of one group sort.
template <int BLOCK, int CAPMAX>
struct SortLds {
    static constexpr int NCS = CAPMAX / 64 + 2;  // match chunks a group overlaps (chunks of >= 64 records)
    static constexpr int NW2 = kSubBins / 2;     // two 16-bit sub-bin counters per word
    uint64_t keys[CAPMAX + 4];  // + four all-ones sentinels after the group's records
    uint32_t nonces[CAPMAX];
    uint32_t start[NW2 + 1];
    uint64_t wave[BLOCK / 64 + 1];
    uint32_t csum[NCS];
};

// Sorts group g into Table 1 with its bucket offsets and, with pcnt, each
// record's pair count (one byte) and (with csum) the counts summed per match
// chunk.  A group over the capacity goes to the overflow list for the
// fallback.  Run by the whole work-group; LDS is free again once every
// thread has returned.
template <int BLOCK, int CAPMAX>
__device__ __forceinline__ void sort_one_group(uint32_t g, const SortArgs &A, SortLds<BLOCK, CAPMAX> &S) {
    constexpr int ITEMS = CAPMAX / BLOCK;
    constexpr int NCS = SortLds<BLOCK, CAPMAX>::NCS;
    static_assert(CAPMAX < 65536 && SortLds<BLOCK, CAPMAX>::NW2 % BLOCK == 0, "packed counters");
    uint64_t *s_keys = S.keys;
    uint32_t *s_nonces = S.nonces;
    uint32_t *s_csum = S.csum;
    uint32_t *s_wave32 = reinterpret_cast<uint32_t *>(S.wave);
    const uint32_t tid = threadIdx.x;
    const uint32_t sb_shift = 64u - A.G - kSubBinBits;
    const uint32_t nbg = 1u << (VXK_BUCKET_BITS - A.G);
    uint64_t *keys = A.keys;
    uint32_t *nonces = A.nonces;
    const GroupIn &in = A.in;
    const uint32_t *gstart = A.gstart;
    const uint32_t G = A.G, cap = A.cap, n_total = A.n_total, cb = A.cb;
    uint32_t *offsets = A.offsets, *ovf_count = A.ovf_count, *ovf_list = A.ovf_list;
    uint8_t *pcnt = A.pcnt;
    unsigned long long *csum = A.csum;
    const uint64_t T = A.T;
    if (g == (1u << G) - 1 && tid == 0) offsets[VXK_NUM_BUCKETS] = n_total;
    const uint32_t lo = gstart[g], n = group_records(in, gstart, g, lo);
    if (in.keys) zero_holes(pcnt, gstart, g, G, lo, n, n_total);
    const uint64_t *src_k = in.keys ? in.keys + in.lo[g] : keys + lo;
    const uint32_t *src_n = in.keys ? in.nonces + in.lo[g] : nonces + lo;
    uint64_t k[ITEMS];
    uint32_t nn[ITEMS];
    if (csum)
        for (uint32_t i = tid; i < (uint32_t)NCS; i += BLOCK) s_csum[i] = 0;  // read after the sort's barriers
    if (n <= cap && n > 0) {
        // Clamped, unconditional loads: a wave issues all before waiting.
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = j * BLOCK + tid;
            const uint32_t ec = e < n ? e : n - 1;
            k[j] = src_k[ec];
            nn[j] = src_n[ec];
        }
    }
    if (n > cap) {
        if (tid == 0) {
            const uint32_t i = atomicAdd(ovf_count, 1u);
            ovf_list[i] = g;
        }
    } else {
        // The LDS sort at the lowest wave priority, the loads before it and
        // the write-out after it at a raised one (issued ahead of the other
        // work-groups' LDS work).
        __builtin_amdgcn_s_setprio(0);
        lds_sort_group<BLOCK, CAPMAX>(k, nn, n, sb_shift, s_keys, s_nonces, S.start, s_wave32);
        __builtin_amdgcn_s_setprio(2);
        // Write the group out, with each record's pair count (one byte):
        // lane-strided records keep LDS reads and stores contiguous; a
        // record tests its next four records with independent reads (no
        // chain of dependent loads) and walks on only past four partners.
        // With csum, every wave also adds its 64 consecutive records'
        // exact counts into the (at most two) match chunks they fall in.
        const uint32_t c_lo = lo >> cb;
        for (uint32_t e0 = 0; e0 < n; e0 += BLOCK) {
            const uint32_t e = e0 + tid;
            uint32_t cnt_e = 0;
            if (e < n) {
                const uint64_t ki = s_keys[e];
                keys[lo + e] = ki;
                nonces[lo + e] = s_nonces[e];
                if (pcnt) {
                    // The partners of record e are the records after it with
                    // a key at most ulim: in its bucket and less than T above
                    // it.  Keys are sorted, so they form a prefix, and the
                    // group's records are followed by all-ones sentinels, which
                    // only a bound of all ones (keys within T of 2^64 in the
                    // last bucket, where every later record is a partner)
                    // would take: that bound counts records instead.
                    const uint64_t bend = ki | ((1ull << 40) - 1u);
                    const uint64_t tl = ki > ~0ull - (T - 1u) ? ~0ull : ki + (T - 1u);
                    const uint64_t ulim = T == 0 ? 0 : (tl < bend ? tl : bend);
                    uint32_t c = 0;
                    if (T != 0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) c += s_keys[e + 1 + r] <= ulim ? 1u : 0u;
                        if (ulim == ~0ull) c = min(c, n - 1u - e);
                        if (c == 4)
                            for (uint32_t j = e + 5; j < n && s_keys[j] <= ulim; ++j) ++c;
                    }
                    pcnt[lo + e] = (uint8_t)min(c, kPairCountEscape);
                    cnt_e = c;
                }
            }
            if (csum) {
                const uint32_t ca = (lo + e0 + (tid & ~63u)) >> cb;  // the wave's first chunk
                const uint32_t va = ((lo + e) >> cb) == ca ? cnt_e : 0u;
                const uint32_t sa = vxd::wave_sum(va), sb = vxd::wave_sum(cnt_e - va);
                if ((tid & 63u) == 0) {
                    if (sa) atomicAdd(&s_csum[ca - c_lo], sa);
                    if (sb) atomicAdd(&s_csum[ca + 1 - c_lo], sb);
                }
            }
        }
        // offsets[b] for the group's buckets: first record with bucket >= b.
        // With at most kSubBinBits bucket bits inside the group they are the
        // top bits of the sub-bin, and a bucket starts where its first
        // sub-bin does (the counting sort's starts, still in S.start);
        // otherwise a binary search over the sorted keys.
        const uint32_t bb = VXK_BUCKET_BITS - G, bfirst = g << bb;
        for (uint32_t bl = tid; bl < nbg; bl += BLOCK) {
            const uint32_t b = bfirst + bl;
            uint32_t a = 0;
            if (bb <= (uint32_t)kSubBinBits) {
                const uint32_t sb = bl << (kSubBinBits - bb);
                a = (S.start[sb >> 1] >> ((sb & 1u) << 4)) & 0xFFFFu;
            } else {
                uint32_t c = n;
                while (a < c) {
                    const uint32_t mid = (a + c) >> 1;
                    if ((uint32_t)(s_keys[mid] >> 40) < b) a = mid + 1; else c = mid;
                }
            }
            offsets[b] = lo + a;
        }
        __syncthreads();
        if (csum && n) {  // the chunks of records [lo, lo + n)
            const uint32_t nch = ((lo + n - 1) >> cb) - c_lo + 1;
            for (uint32_t i = tid; i < nch; i += BLOCK)
                if (s_csum[i]) atomicAdd(&csum[c_lo + i], (unsigned long long)s_csum[i]);
        }
    }
}

// Persistent: each work-group takes groups of [g0, g0 + gcount) from a
// ticket counter (*ticket, zero at launch) until none is left, so work-groups
// that start late -- while another stream's kernel holds part of the device
// -- simply take fewer groups.  The kernel is kept at 64 VGPRs or fewer so
// that four work-groups share each CU; their phases interleave, which hides
// each one's global loads behind the others' LDS work (better, measured,
// than prefetching into registers at fewer work-groups per CU).
template <int BLOCK, int CAPMAX>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(CAPMAX <= kGroupCapFast ? 8 : 1))) void k_groupsort(SortArgs A, uint32_t g0, uint32_t gcount,
                                                                                                                          uint32_t *__restrict__ ticket) {
    __shared__ SortLds<BLOCK, CAPMAX> S;
    __shared__ uint32_t s_tk[2];  // alternate, so a slow reader never sees the next ticket
    const uint32_t tid = threadIdx.x;
    __builtin_amdgcn_s_setprio(2);
    for (uint32_t it = 0;; ++it) {
        if (tid == 0) s_tk[it & 1] = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t t = s_tk[it & 1];
        if (t >= gcount) break;
        sort_one_group<BLOCK, CAPMAX>(g0 + t, A, S);
    }
}

// Groups larger than the LDS capacity: rank sort against LDS-staged tiles of
// the group (copied to scratch first), then bucket offsets by binary search
// and the pair count in global memory.  Groups above fb_max set a status bit
// and stay unsorted.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_group_fallback(
    uint64_t *keys, uint32_t *nonces, GroupIn in, uint64_t *scr_keys,
    uint32_t *scr_nonces, const uint32_t *__restrict__ gstart, uint32_t G,
    uint32_t *__restrict__ offsets, const uint32_t *__restrict__ ovf_count,
    const uint32_t *__restrict__ ovf_list, uint32_t fb_max, uint32_t *__restrict__ status,
    uint64_t T, uint8_t *__restrict__ pcnt, unsigned long long *__restrict__ csum, uint32_t cb) {
    __shared__ uint64_t s_k[BLOCK];
    __shared__ uint32_t s_n[BLOCK];
    const uint32_t tid = threadIdx.x;
    const uint32_t cnt = *ovf_count;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint32_t g = ovf_list[i];
        const uint32_t lo = gstart[g], n = group_records(in, gstart, g, lo);
        if (n > fb_max) {
            if (tid == 0) atomicOr(status, (uint32_t)VXK_DEV_STATUS_GROUP_TOO_LARGE);
            continue;
        }
        // The records to rank: the input regions, or (in place) a copy in
        // the scratch arrays.
        const uint64_t *sk;
        const uint32_t *sn;
        if (in.keys) {
            sk = in.keys + in.lo[g];
            sn = in.nonces + in.lo[g];
        } else {
            for (uint32_t e = tid; e < n; e += BLOCK) {
                scr_keys[lo + e] = keys[lo + e];
                scr_nonces[lo + e] = nonces[lo + e];
            }
            sk = scr_keys + lo;
            sn = scr_nonces + lo;
        }
        __syncthreads();
        for (uint32_t e0 = 0; e0 < n; e0 += BLOCK) {
            const uint32_t e = e0 + tid;
            const bool valid = e < n;
            uint64_t mk = 0;
            uint32_t mn = 0, r = 0;
            if (valid) {
                mk = sk[e];
                mn = sn[e];
            }
            for (uint32_t t0 = 0; t0 < n; t0 += BLOCK) {
                __syncthreads();
                if (t0 + tid < n) {
                    s_k[tid] = sk[t0 + tid];
                    s_n[tid] = sn[t0 + tid];
                }
                __syncthreads();
                const uint32_t m = min((uint32_t)BLOCK, n - t0);
                if (valid)
                    for (uint32_t x = 0; x < m; ++x) r += rec_less(s_k[x], s_n[x], mk, mn);
            }
            if (valid) {
                keys[lo + r] = mk;
                nonces[lo + r] = mn;
            }
        }
        __syncthreads();
        const uint32_t nbg = 1u << (VXK_BUCKET_BITS - G);
        const uint32_t bfirst = g << (VXK_BUCKET_BITS - G);
        for (uint32_t bl = tid; bl < nbg; bl += BLOCK) {
            const uint32_t b = bfirst + bl;
            uint32_t a = 0, c = n;
            while (a < c) {
                const uint32_t mid = (a + c) >> 1;
                if ((uint32_t)(keys[lo + mid] >> 40) < b) a = mid + 1; else c = mid;
            }
            offsets[b] = lo + a;
        }
        if (pcnt && n) {
            const uint32_t per = (n + BLOCK - 1) / BLOCK;
            const uint32_t r0 = min(tid * per, n), r1 = min(r0 + per, n);
            pairs_in_range(keys + lo, r0, r1, n, T, pcnt + lo, csum, cb, lo);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Match over fixed chunks of Table 1 (chunk c = records [c << cb, (c+1) << cb)).
// A record's pairs are owned by its chunk even when the partner lies in the
// next chunk; pairs never cross a bucket, so the forward scan stops at the
// bucket's end.
// ---------------------------------------------------------------------------

// Pair count per chunk and per record (used when the sort did not provide
// them).
template <int BLOCK, int MCAP>
__global__ __launch_bounds__(BLOCK) void k_match_count(const uint64_t *__restrict__ keys,
                                                       uint32_t n_total, uint32_t cb, uint64_t T,
                                                       uint64_t *__restrict__ counts,
                                                       uint8_t *__restrict__ pcnt) {
    __shared__ uint64_t s_keys[MCAP];
    __shared__ uint64_t s_wave[BLOCK / 64 + 1];
    const uint32_t tid = threadIdx.x;
    const uint32_t nchunks = (n_total + (1u << cb) - 1) >> cb;
    for (uint32_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
        const uint32_t c = ci << cb;
        const uint32_t m = min(1u << cb, n_total - c);
        for (uint32_t e = tid; e < m; e += BLOCK) s_keys[e] = keys[c + e];
        __syncthreads();
        uint64_t total = 0;
        for (uint32_t e = tid; e < m; e += BLOCK) {
            const uint64_t ki = s_keys[e];
            const uint32_t bi = (uint32_t)(ki >> 40);
            uint32_t mine = 0;
            for (uint32_t j = c + e + 1; j < n_total; ++j) {
                const uint64_t kj = (j - c < m) ? s_keys[j - c] : keys[j];
                if ((uint32_t)(kj >> 40) != bi || kj - ki >= T) break;
                ++mine;
            }
            pcnt[c + e] = (uint8_t)min(mine, kPairCountEscape);
            total += mine;
        }
        total = vxd::block_sum<BLOCK>(total, s_wave);
        if (tid == 0) counts[ci] = total;
    }
}

// A value the program knows to be equal in every lane (e.g. loaded from one
// LDS address), moved to scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Pairs owned by record i of the sorted Table 1 (global walk; used for
// records whose count byte is the escape value).
__device__ __forceinline__ uint32_t pairs_after_global(const uint64_t *keys, uint32_t i, uint32_t n_total,
                                                       uint64_t T) {
    const uint64_t ki = keys[i];
    const uint32_t bi = (uint32_t)(ki >> 40);
    uint32_t c = 0;
    for (uint32_t j = i + 1; j < n_total; ++j) {
        const uint64_t kj = keys[j];
        if ((uint32_t)(kj >> 40) != bi || kj - ki >= T) break;
        ++c;
    }
    return c;
}

// Match chunks owned by a range of Table-1 records: a chunk belongs to the
// range holding its last record, so chunks [*r_lo >> cb, *r_hi >> cb) (to
// the end for the last range) -- once every record before *r_hi is sorted,
// these chunks and all their partners are final.  No range (r_lo NULL): all.
__device__ __forceinline__ void chunk_range(const uint32_t *r_lo, const uint32_t *r_hi, uint32_t last,
                                            uint32_t cb, uint32_t nchunks, uint32_t &c0, uint32_t &c1) {
    if (!r_lo) {
        c0 = 0;
        c1 = nchunks;
        return;
    }
    c0 = min(*r_lo >> cb, nchunks);
    c1 = last ? nchunks : min(*r_hi >> cb, nchunks);
    if (c1 < c0) c1 = c0;
}

// Table-2 pair count of every match chunk (of a record range) from the
// per-record count bytes: one wave per chunk, 16-byte loads, no barriers.
// Escaped bytes are recounted from the keys.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_chunk_sums(const uint8_t *__restrict__ pcnt,
                                                      const uint64_t *__restrict__ keys, uint32_t n_total,
                                                      uint32_t cb, uint64_t T, uint64_t *__restrict__ counts,
                                                      const uint32_t *r_lo, const uint32_t *r_hi,
                                                      uint32_t last) {
    constexpr int WPB = BLOCK / 64;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nchunks = (n_total + (1u << cb) - 1) >> cb;
    uint32_t c0, c1;
    chunk_range(r_lo, r_hi, last, cb, nchunks, c0, c1);
    for (uint32_t ci = c0 + blockIdx.x * WPB + threadIdx.x / 64; ci < c1; ci += gridDim.x * WPB) {
        const uint32_t c = ci << cb, m = min(1u << cb, n_total - c);
        // 16 count bytes per lane and load (a chunk starts on a 64-byte
        // boundary of the 256-byte aligned count array), then the chunk's
        // last m mod 16 bytes one by one.
        const uint32_t n16 = m >> 4;
        const uint4 *v16 = reinterpret_cast<const uint4 *>(pcnt + c);
        uint64_t sum = 0;
        for (uint32_t w = lane; w < n16; w += 64) {
            const uint4 v = v16[w];
            const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t b = (q[k] >> (8 * i)) & 0xffu;
                    sum += b == kPairCountEscape ? pairs_after_global(keys, c + 16 * w + 4 * k + i, n_total, T) : b;
                }
            }
        }
        for (uint32_t e = (n16 << 4) + lane; e < m; e += 64) {
            const uint32_t b = pcnt[c + e];
            sum += b == kPairCountEscape ? pairs_after_global(keys, c + e, n_total, T) : b;
        }
        sum = vxd::wave_sum(sum);
        if (lane == 0) counts[ci] = sum;
    }
}

// Table-2 bases of the chunks of a record range: bases = *acc + exclusive
// prefix of the counts; *acc then grows by the range's total, and the last
// range stores the grand total in *t2_count.  One work-group; ranges are
// scanned in order on one stream.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_scan_range(const uint64_t *__restrict__ counts,
                                                      uint64_t *__restrict__ bases, uint32_t n_total,
                                                      uint32_t cb, const uint32_t *r_lo, const uint32_t *r_hi,
                                                      uint32_t last, uint64_t *acc, uint64_t *t2_count) {
    __shared__ uint64_t s_wave[BLOCK / 64 + 1];
    const uint32_t nchunks = (n_total + (1u << cb) - 1) >> cb;
    uint32_t c0, c1;
    chunk_range(r_lo, r_hi, last, cb, nchunks, c0, c1);
    const uint32_t n = c1 - c0;
    const uint32_t per = (n + BLOCK - 1) / BLOCK;
    const uint32_t a = c0 + min(threadIdx.x * per, n), b = c0 + min((threadIdx.x + 1) * per, n);
    uint64_t mine = 0;
    for (uint32_t c = a; c < b; ++c) mine += counts[c];
    uint64_t total;
    uint64_t run = vxd::block_exclusive_scan<BLOCK>(mine, s_wave, &total) + *acc;
    for (uint32_t c = a; c < b; ++c) {
        const uint64_t v = counts[c];
        bases[c] = run;
        run += v;
    }
    __syncthreads();  // every thread has read *acc
    if (threadIdx.x == 0) {
        const uint64_t t = *acc + total;
        *acc = t;
        if (last) *t2_count = t;
    }
}

// Match + Table-2 hash.  A persistent work-group takes match chunks from a
// ticket counter (*ticket, zero at launch).  The pair count of every record
// was stored as one byte by the kernel that counted the chunks (the group
// sort, or the match count), so keys are read only for escaped counts.
// Per chunk:
//  * thread t owns records 4t .. 4t+3 (one 32-bit load of their count
//    bytes); a work-group scan turns the counts into canonical Table-2 slots
//    and each record's first slot is kept in LDS;
//  * the chunk's slots are taken in windows of SLOTS (one window unless the
//    keys are crowded): every record writes its index into the LDS word of
//    each of its slots in the window, then slot q is hashed by lane
//    q mod BLOCK -- every lane hashes the same number of pairs (+-1) and a
//    wave's stores fill one contiguous 1 KiB run of Table 2.
// Table-2 index = chunk base + slot.  The next chunk's nonces and counts are
// loaded into registers while the current one is worked on.
// A Table-1 nonce read from global memory, kept out of line (see its use in
// k_match_emit).
__device__ __noinline__ uint32_t load_nonce_slow(const uint32_t *nonces, uint32_t i) { return nonces[i]; }


template <int BLOCK, int MCAP, int SLOTS>
struct MatchLds {
    uint32_t nonces[MCAP];
    uint64_t first[MCAP];  // first Table-2 slot of each record (chunk-relative)
    uint32_t slot[SLOTS];  // record owning each slot of the window
    uint64_t wave[BLOCK / 64 + 1];
};

// Loads chunk ci's nonces (pn, lane-strided) and thread t's word of count
// bytes (records 4t .. 4t+3).
template <int BLOCK, int ITEMS>
__device__ __forceinline__ void match_load(const MatchArgs &A, uint32_t ci, uint32_t (&pn)[ITEMS], uint32_t &pc) {
    const uint32_t tid = threadIdx.x;
    const uint32_t c = ci << A.cb, m = min(1u << A.cb, A.n_total - c);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = tid + i * BLOCK;
        if (e < m) pn[i] = A.nonces[c + e];
    }
    if (tid * ITEMS < m) pc = *reinterpret_cast<const uint32_t *>(A.pcnt + c + tid * ITEMS);
}

// Match + Table-2 hash of chunk ci, whose nonces and count word the caller
// loaded (match_load).  `between` runs once the chunk's counts are scanned
// (the persistent kernel loads the next chunk there).  Run by the whole
// work-group; LDS is free again once every thread has returned.
template <int BLOCK, int MCAP, int SLOTS, typename F>
__device__ __forceinline__ void match_one_chunk(uint32_t ci, const MatchArgs &A, MatchLds<BLOCK, MCAP, SLOTS> &S,
                                                const uint32_t (&pn)[MCAP / BLOCK], uint32_t pc, F between) {
    constexpr int ITEMS = MCAP / BLOCK;
    static_assert(ITEMS == 4, "one 32-bit word of count bytes per thread");
    uint32_t *s_nonces = S.nonces;
    uint64_t *s_first = S.first;
    uint32_t *s_slot = S.slot;
    const uint32_t tid = threadIdx.x;
    const uint32_t e0 = tid * ITEMS;
    const uint32_t n_total = A.n_total;
    const uint32_t c = ci << A.cb, m = min(1u << A.cb, n_total - c);
    Key key;
#pragma unroll
    for (int w = 0; w < 8; ++w) key.w[w] = A.key[w];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = tid + i * BLOCK;
        if (e < m) s_nonces[e] = pn[i];
    }
    // The count, scan and slot expansion (barriers, LDS) at a raised wave
    // priority, the hash loop at the lowest: a work-group between two
    // barriers then holds the others' hashing up less.
    __builtin_amdgcn_s_setprio(2);
    const uint32_t cw = pc;
    const uint64_t base = A.chunk_base[ci];
    uint32_t cnt[ITEMS];
    uint64_t mine = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        uint32_t cc = 0;
        if (e0 + i < m) {
            cc = (cw >> (8 * i)) & 0xffu;
            if (cc == kPairCountEscape) cc = pairs_after_global(A.keys, c + e0 + i, n_total, A.T);
        }
        cnt[i] = cc;
        mine += cc;
    }
    uint64_t ctot;
    const uint64_t run = vxd::block_exclusive_scan<BLOCK>(mine, S.wave, &ctot);
    ctot = uniform_u64(ctot);  // same in every lane: keep it in scalar registers
    between();
    // A pair-free chunk skips the LDS writes below (it has no barrier after
    // them before the next chunk).
    if (ctot == 0) return;
    uint4 *out = A.t2 + base;
    const uint64_t cap = A.cap;
    if (ctot <= SLOTS) {
        // One window (every chunk of BLAKE3 keys): slots fit 32 bits, and a
        // chunk whose slots all fit Table 2 skips the per-pair check.
        uint32_t *s_first32 = reinterpret_cast<uint32_t *>(s_first);
        uint32_t r = (uint32_t)run;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            // A record's slots: the first four as masked stores at fixed
            // offsets (a wave would otherwise loop as often as its largest
            // count), a loop only for the rare record with more.
            s_first32[e0 + i] = r;
            uint32_t *dst = s_slot + r;
            const uint32_t ni = cnt[i], val = e0 + i;
            if (ni > 0) dst[0] = val;
            if (ni > 1) dst[1] = val;
            if (ni > 2) dst[2] = val;
            if (ni > 3) dst[3] = val;
            for (uint32_t q = 4; q < ni; ++q) dst[q] = val;
            r += ni;
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        const uint32_t nq = (uint32_t)ctot;
        auto pair = [&](uint32_t qr, uint32_t &na, uint32_t &nb) {
            const uint32_t e = s_slot[qr];
            const uint32_t j = e + 1 + qr - s_first32[e];
            na = s_nonces[e];
            // The partner is almost always in this chunk's LDS copy; an
            // out-of-line load for the rest keeps the compiler from merging
            // the two into a generic (flat) load per pair.
            if (__builtin_expect(j < m, 1))
                nb = s_nonces[j];
            else
                nb = load_nonce_slow(A.nonces, c + j);
        };
        if (base + ctot <= cap) {
#pragma unroll 1
            for (uint32_t qr = tid; qr < nq; qr += BLOCK) {
                uint32_t na, nb;
                pair(qr, na, nb);
                const uint64_t h = vxd::h2(key, na, nb);
                out[qr] = make_uint4(na, nb, (uint32_t)h, (uint32_t)(h >> 32));
            }
        } else {
#pragma unroll 1
            for (uint32_t qr = tid; qr < nq; qr += BLOCK) {
                uint32_t na, nb;
                pair(qr, na, nb);
                const uint64_t h = vxd::h2(key, na, nb);
                if (base + qr < cap) out[qr] = make_uint4(na, nb, (uint32_t)h, (uint32_t)(h >> 32));
            }
        }
        __syncthreads();
        return;
    }
    const uint64_t run_end = run + mine;
    {
        const uint64_t w1 = SLOTS;
        uint64_t r = run;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            s_first[e0 + i] = r;
            const uint64_t hi = r + cnt[i] < w1 ? r + cnt[i] : w1;
            for (uint64_t q = r; q < hi; ++q) s_slot[q] = e0 + i;
            r += cnt[i];
        }
    }
#pragma unroll 1
    for (uint64_t w0 = 0; w0 < ctot;) {
        const uint64_t w1 = w0 + SLOTS < ctot ? w0 + SLOTS : ctot;
        __syncthreads();
        const uint32_t nq = (uint32_t)(w1 - w0);
#pragma unroll 1
        for (uint32_t qr = tid; qr < nq; qr += BLOCK) {
            const uint32_t e = s_slot[qr];
            const uint64_t q = w0 + qr;
            const uint32_t j = e + 1 + (uint32_t)(q - s_first[e]);
            const uint32_t na = s_nonces[e];
            // The partner is almost always in this chunk's LDS copy; an
            // out-of-line load for the rest keeps the compiler from merging
            // the two into a generic (flat) load per pair.
            uint32_t nb;
            if (__builtin_expect(j < m, 1))
                nb = s_nonces[j];
            else
                nb = load_nonce_slow(A.nonces, c + j);
            const uint64_t h = vxd::h2(key, na, nb);
            if (base + q < cap) out[q] = make_uint4(na, nb, (uint32_t)h, (uint32_t)(h >> 32));
        }
        __syncthreads();
        w0 = w1;
        if (w0 < ctot) {  // next window (crowded keys only): runs from LDS
            const uint64_t w2 = w0 + SLOTS < ctot ? w0 + SLOTS : ctot;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint64_t f = s_first[e0 + i];
                const uint64_t g = i + 1 < ITEMS ? s_first[e0 + i + 1] : run_end;
                const uint64_t lo = f > w0 ? f : w0;
                const uint64_t hi = g < w2 ? g : w2;
                for (uint64_t q = lo; q < hi; ++q) s_slot[q - w0] = e0 + i;
            }
        }
    }
}

template <int BLOCK, int MCAP, int SLOTS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_match_emit(MatchArgs A, const uint32_t *r_lo, const uint32_t *r_hi,
                                                      uint32_t last, uint32_t *__restrict__ ticket) {
    constexpr int ITEMS = MCAP / BLOCK;
    __shared__ MatchLds<BLOCK, MCAP, SLOTS> S;
    __shared__ uint32_t s_tk[2];  // alternate, so a slow reader never sees the next ticket
    const uint32_t tid = threadIdx.x;
    uint32_t c0, nchunks;  // this launch's chunks: [c0, nchunks)
    chunk_range(r_lo, r_hi, last, A.cb, (A.n_total + (1u << A.cb) - 1) >> A.cb, c0, nchunks);
    if (tid == 0) s_tk[1] = atomicAdd(ticket, 1u);
    __syncthreads();
    uint32_t ci = c0 + s_tk[1];
    if (ci >= nchunks) return;
    uint32_t pn[ITEMS], pc = 0;
    match_load<BLOCK, ITEMS>(A, ci, pn, pc);
    for (uint32_t it = 0;; ++it) {
        if (tid == 0) s_tk[it & 1] = atomicAdd(ticket, 1u);  // the next chunk, read after the scan
        uint32_t cur[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) cur[i] = pn[i];
        const uint32_t cpc = pc;
        uint32_t nci = 0;
        bool more = false;
        // Prefetch the next chunk into registers while this one is hashed.
        match_one_chunk<BLOCK, MCAP, SLOTS>(ci, A, S, cur, cpc, [&]() {
            nci = c0 + s_tk[it & 1];
            more = nci < nchunks;
            if (more) match_load<BLOCK, ITEMS>(A, nci, pn, pc);
        });
        if (!more) break;
        ci = nci;
    }
}

// ---------------------------------------------------------------------------
// One persistent launch of a software-pipelined plot (or batch of plots):
// items of up to four kinds -- hash sub-tiles (H), partition-pass sub-tiles
// (P), group sorts (S) and match chunks (M) -- from slices whose inputs
// earlier launches finished (stream order makes them visible; no item
// waits on another).  Work-groups take items from one ticket counter, the
// kinds interleaved in proportion to their numbers, so that the vector-ALU
// work (hash, match) and the memory and LDS work (passes, sort) of
// different slices share every CU.  The kinds share one LDS area, so every
// item starts behind a barrier; the filing counters have their own.
// ---------------------------------------------------------------------------

// The four kinds of k_pipe items, each out of line so that none keeps
// another's values in registers.
template <int BLOCK>
struct PipeLds {
    static constexpr int CAP = kGroupCapFast;
    union Area {
        struct {
            uint64_t keys[kPipeSub];
            uint32_t non[kPipeSub];
        } f;
        SortLds<BLOCK, CAP> s;
        MatchLds<BLOCK, kMatchCap, kMatchSlots> m;
    } a;
    uint32_t cnt[1 << kPipeMaxBits];
    uint32_t pos[(1 << kPipeMaxBits) + 1];
    uint2 dst[1 << kPipeMaxBits];
};

template <int BLOCK>
__device__ __noinline__ void pipe_hash(const HashSliceDesc &H, uint32_t x, PipeLds<BLOCK> &S) {
    constexpr int FI = kPipeSub / BLOCK;
    uint64_t k[FI];
    uint32_t nv[FI];
    const uint32_t m = hash_subtile<BLOCK, FI>(H, x, k, nv);
    file_records<BLOCK, FI, 1 << kPipeMaxBits>(k, nv, m, 64u - H.bits, H.bits, H.fill, 0, H.R, H.keys, H.nonces,
                                                   H.status, S.a.f.keys, S.a.f.non, S.cnt, S.pos, S.dst, [] {});
}

template <int BLOCK>
__device__ __noinline__ void pipe_pass(const PassSliceDesc &P, uint32_t x, PipeLds<BLOCK> &S) {
    constexpr int FI = kPipeSub / BLOCK;
    uint64_t k[FI];
    uint32_t nv[FI], r;
    const uint32_t m = load_subtile<BLOCK, FI>(P, x, k, nv, &r);
    file_records<BLOCK, FI, 1 << kPipeMaxBits>(k, nv, m, P.shift, P.bits, P.out_fill, (P.r0 + r) << P.bits,
                                                   P.R_out, P.out_keys, P.out_nonces, P.status, S.a.f.keys,
                                                   S.a.f.non, S.cnt, S.pos, S.dst, [] {});
}

template <int BLOCK>
__device__ __noinline__ void pipe_sort(const PipeSortDesc &D, uint32_t x, PipeLds<BLOCK> &S) {
    sort_one_group<BLOCK, PipeLds<BLOCK>::CAP>(D.g0 + x, D.a, S.a.s);
}

template <int BLOCK>
__device__ __noinline__ void pipe_match(const PipeMatchDesc &M, uint32_t x, PipeLds<BLOCK> &S) {
    uint32_t c0, c1;
    chunk_range(M.r_lo, M.r_hi, M.last, M.a.cb, (M.a.n_total + (1u << M.a.cb) - 1) >> M.a.cb, c0, c1);
    const uint32_t ci = c0 + x;
    if (ci >= c1) return;  // the item count is an upper bound
    uint32_t pn[kMatchCap / BLOCK], pc = 0;
    match_load<BLOCK, kMatchCap / BLOCK>(M.a, ci, pn, pc);
    match_one_chunk<BLOCK, kMatchCap, kMatchSlots>(ci, M.a, S.a.m, pn, pc, [] {});
}

// The launch's list is read from device memory (k_store_list wrote it), so
// the items' descriptors are passed on by address without copies.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_pipe(const PipeList *__restrict__ Lp,
                                                                                uint32_t *__restrict__ ticket) {
    const PipeList &L = *Lp;
    __shared__ PipeLds<BLOCK> S;
    __shared__ uint32_t s_tk[2];  // alternate, so a slow reader never sees the next ticket
    const uint32_t tid = threadIdx.x;
    const uint64_t NT = (uint64_t)L.items[0] + L.items[1] + L.items[2] + L.items[3];
    if (tid < (1u << kPipeMaxBits)) S.cnt[tid] = 0;
    for (uint32_t it = 0;; ++it) {
        if (tid == 0) s_tk[it & 1] = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint64_t t = s_tk[it & 1];
        if (t >= NT) break;
        uint64_t i1, i2, i3;
        uint32_t d = 0;
        if (take_first(t, L.frac[0], i1)) {
            uint32_t x = (uint32_t)i1;
            while (d + 1 < L.n[0] && x >= L.h[d].items) x -= L.h[d].items, ++d;
            pipe_hash<BLOCK>(L.h[d], x, S);
        } else if (take_first(i1, L.frac[1], i2)) {
            uint32_t x = (uint32_t)i2;
            while (d + 1 < L.n[1] && x >= L.p[d].items) x -= L.p[d].items, ++d;
            pipe_pass<BLOCK>(L.p[d], x, S);
        } else if (take_first(i2, L.frac[2], i3)) {
            uint32_t x = (uint32_t)i3;
            while (d + 1 < L.n[2] && x >= L.s[d].items) x -= L.s[d].items, ++d;
            pipe_sort<BLOCK>(L.s[d], x, S);
        } else {
            uint32_t x = (uint32_t)i3;
            while (d + 1 < L.n[3] && x >= L.m[d].items) x -= L.m[d].items, ++d;
            pipe_match<BLOCK>(L.m[d], x, S);
        }
    }
}

// ---------------------------------------------------------------------------
// Fused group sort + match + Table-2 hash (the plot's tail; paper sec. III-A
// fuses the sort and the match of a bucket in one block).
//
// A persistent work-group takes sort groups in increasing order from a
// ticket counter.  For group g it
//  1. gathers the group's records from its partition region (or reads them
//     in place), sorts them in LDS (lds_sort_group) and writes the group's
//     Table-1 slice and bucket offsets;
//  2. counts each record's pairs from the sorted keys in LDS -- exactly,
//     because partners never leave a group (groups end at bucket
//     boundaries);
//  3. publishes the group's pair total and obtains its Table-2 base with a
//     decoupled look-back over the totals of the groups before it
//     (single-pass scan, Merrill and Garland 2016): it publishes its own
//     total first, then sums published totals backwards until it meets a
//     published inclusive prefix.  Tickets are handed out in order to
//     running work-groups and every work-group publishes its total before it
//     waits, so the waits always end; the wait is still bounded and sets a
//     status bit if the bound is hit;
//  4. expands the pairs into LDS (each slot names its first record) and
//     hashes them one pair per lane, writing Table 2 at base + slot.
// The work-groups resident on a CU are at different steps, so the sorts'
// memory and LDS work runs beside the hashes' vector work.  Table 1 is read
// once (from the regions) and never read back, and only the pair totals
// cross work-groups.  Groups above the LDS capacity are sorted and matched by
// the same work-group in global memory (slow path; never taken by BLAKE3 keys
// at the default group bits).
// ---------------------------------------------------------------------------

constexpr uint64_t kLbAgg = 1ull << 62;     // word holds the group's own count
constexpr uint64_t kLbPrefix = 2ull << 62;  // word holds the inclusive prefix
constexpr uint64_t kLbValue = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Run by the whole work-group.  Returns (in every thread) the sum of the
// counts of groups [0, g).  Thread t inspects group j - t, so one round
// covers BLOCK predecessors -- about the number of groups in flight, which is
// how far back the nearest published inclusive prefix usually is.  A round
// consumes the window up to the first group that is not yet published or
// that carries an inclusive prefix.
template <int BLOCK>
__device__ uint64_t lookback(const uint64_t *words, uint32_t g, uint32_t spin_limit,
                             uint32_t *dev_status, uint32_t *s_first, uint64_t *s_wave) {
    constexpr int NW = BLOCK / 64;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid / 64u;
    uint64_t prefix = 0;
    int64_t j = (int64_t)g - 1;
    uint32_t spins = 0;
    while (j >= 0) {
        const int64_t idx = j - (int64_t)tid;
        const uint64_t v = idx >= 0 ? lb_load(&words[idx]) : kLbPrefix;
        const uint64_t flag = v & ~kLbValue;
        const uint64_t not_ready = __ballot(flag == 0);
        const uint64_t pref = __ballot(flag == kLbPrefix);
        if (lane == 0) {
            s_first[wid] = not_ready ? (uint32_t)__builtin_ctzll(not_ready) : 64u;
            s_first[NW + wid] = pref ? (uint32_t)__builtin_ctzll(pref) : 64u;
        }
        __syncthreads();
        uint32_t first_nr = BLOCK, first_pf = BLOCK;
#pragma unroll
        for (int w = NW - 1; w >= 0; --w) {
            if (s_first[w] < 64u) first_nr = w * 64 + s_first[w];
            if (s_first[NW + w] < 64u) first_pf = w * 64 + s_first[NW + w];
        }
        const uint32_t take = first_pf < first_nr ? first_pf + 1 : first_nr;
        prefix += vxd::block_sum<BLOCK>(tid < take ? (uint64_t)(v & kLbValue) : (uint64_t)0, s_wave);
        if (first_pf < first_nr) break;
        j -= take;
        if (take == 0) {
            // Bounded wait.  After any timeout every later look-back gives up
            // at once, so one failure cannot chain into long waits.
            const uint32_t st = __hip_atomic_load(dev_status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (++spins > spin_limit || (st & VXK_DEV_STATUS_LOOKBACK_TIMEOUT)) {
                if (tid == 0) atomicOr(dev_status, (uint32_t)VXK_DEV_STATUS_LOOKBACK_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    return prefix;
}

// Oversized group (n > the LDS capacity): rank sort in global memory, the
// records compared in LDS-staged tiles of CAPMAX records (s_keys / s_nonces),
// written to keys / nonces [lo, lo + n), then the group's bucket offsets.
// src: the group's records (its region, or a scratch copy).  All threads
// call it; it ends with a barrier.
template <int BLOCK, int CAPMAX>
__device__ void slow_sort_group(const uint64_t *src_k, const uint32_t *src_n, uint32_t n, uint64_t *keys,
                                uint32_t *nonces, uint32_t lo, uint32_t g, uint32_t G, uint32_t *offsets,
                                uint64_t *s_keys, uint32_t *s_nonces) {
    const uint32_t tid = threadIdx.x;
    for (uint32_t e0 = 0; e0 < n; e0 += BLOCK) {
        const uint32_t e = e0 + tid;
        const bool valid = e < n;
        uint64_t mk = 0;
        uint32_t mn = 0, r = 0;
        if (valid) {
            mk = src_k[e];
            mn = src_n[e];
        }
        for (uint32_t t0 = 0; t0 < n; t0 += CAPMAX) {
            const uint32_t m = min((uint32_t)CAPMAX, n - t0);
            __syncthreads();
            for (uint32_t x = tid; x < m; x += BLOCK) {
                s_keys[x] = src_k[t0 + x];
                s_nonces[x] = src_n[t0 + x];
            }
            __syncthreads();
            if (valid)
                for (uint32_t x = 0; x < m; ++x) r += rec_less(s_keys[x], s_nonces[x], mk, mn);
        }
        if (valid) {
            keys[lo + r] = mk;
            nonces[lo + r] = mn;
        }
    }
    __syncthreads();
    const uint32_t nbg = 1u << (VXK_BUCKET_BITS - G);
    const uint32_t bfirst = g << (VXK_BUCKET_BITS - G);
    for (uint32_t bl = tid; bl < nbg; bl += BLOCK) {
        uint32_t a = 0, c = n;
        while (a < c) {
            const uint32_t mid = (a + c) >> 1;
            if ((uint32_t)(keys[lo + mid] >> 40) < bfirst + bl) a = mid + 1; else c = mid;
        }
        offsets[bfirst + bl] = lo + a;
    }
    __syncthreads();
}

template <int BLOCK, int CAPMAX, int SLOTS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_group_match(
    Key key, uint64_t *__restrict__ keys, uint32_t *__restrict__ nonces, GroupIn in,
    uint64_t *__restrict__ scr_keys, uint32_t *__restrict__ scr_nonces, const uint32_t *__restrict__ gstart,
    uint32_t G, uint32_t cap, uint32_t *__restrict__ offsets, uint32_t n_total, uint64_t T,
    uint32_t *__restrict__ ticket, uint64_t *__restrict__ words, uint32_t *__restrict__ dev_status,
    uint4 *__restrict__ t2, uint64_t t2cap, uint64_t *__restrict__ t2_count, uint32_t spin_limit,
    uint32_t fb_max) {
    constexpr int ITEMS = CAPMAX / BLOCK;
    constexpr int NW2 = kSubBins / 2;
    static_assert(CAPMAX % BLOCK == 0 && CAPMAX < 65536, "records are indexed by 16 bits");
    static_assert(CAPMAX * 4 + SLOTS * 2 <= CAPMAX * 8, "first slots and the slot window fit the key area");
    static_assert(CAPMAX <= 2 * (NW2 + 1), "16-bit pair counts fit the sub-bin area");
    __shared__ uint64_t s_keys[CAPMAX];      // steps 1-2: sorted keys; step 4: s_first + s_slot
    __shared__ uint32_t s_nonces[CAPMAX];
    __shared__ uint32_t s_start[NW2 + 1];    // step 1: sub-bin counters; steps 2-3: s_cnt
    __shared__ uint64_t s_wave[BLOCK / 64 + 1];
    __shared__ uint32_t s_lb[2 * (BLOCK / 64)];
    __shared__ uint32_t s_tk[2];  // alternate, so a slow reader never sees the next ticket
    uint32_t *s_wave32 = reinterpret_cast<uint32_t *>(s_wave);
    uint16_t *s_cnt = reinterpret_cast<uint16_t *>(s_start);   // pairs owned by each sorted record
    uint32_t *s_first = reinterpret_cast<uint32_t *>(s_keys);  // first slot of each record
    uint16_t *s_slot = reinterpret_cast<uint16_t *>(s_keys) + 2 * CAPMAX;  // record of each window slot
    const uint32_t tid0 = threadIdx.x;
    const uint32_t ngroups = 1u << G;
    const uint32_t sb_shift = 64u - G - kSubBinBits;
    const uint32_t nbg = 1u << (VXK_BUCKET_BITS - G);
    if (blockIdx.x == 0 && tid0 == 0) offsets[VXK_NUM_BUCKETS] = n_total;
    for (uint32_t it = 0;; ++it) {
        // Opaque per group, so that the compiler recomputes thread-derived
        // addresses instead of holding them in registers across the loop (the
        // kernel then fits 80 VGPRs, three work-groups per CU).
        uint32_t tid = tid0;
        asm volatile("" : "+v"(tid));
        if (tid == 0) s_tk[it & 1] = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t g = s_tk[it & 1];
        if (g >= ngroups) break;
        const uint32_t lo = gstart[g], n = group_records(in, gstart, g, lo);
        const uint64_t *src_k = in.keys ? in.keys + in.lo[g] : keys + lo;
        const uint32_t *src_n = in.keys ? in.nonces + in.lo[g] : nonces + lo;
        const bool fast = n <= cap;
        uint64_t mine = 0;  // pairs owned by this thread's records
        if (fast) {
            uint64_t k[ITEMS];
            uint32_t nn[ITEMS];
            if (n > 0) {
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) {
                    const uint32_t e = j * BLOCK + tid;
                    const uint32_t ec = e < n ? e : n - 1;
                    k[j] = src_k[ec];
                    nn[j] = src_n[ec];
                }
            }
            lds_sort_group<BLOCK, CAPMAX>(k, nn, n, sb_shift, s_keys, s_nonces, s_start, s_wave32);
            // Write the group out and count each record's pairs: lane-strided
            // records keep LDS and global accesses contiguous; a record tests
            // its next four records with independent reads and walks on only
            // past four partners.
            for (uint32_t e = tid; e < n; e += BLOCK) {
                const uint64_t ki = s_keys[e];
                keys[lo + e] = ki;
                nonces[lo + e] = s_nonces[e];
                const uint32_t bi = (uint32_t)(ki >> 40);
                uint64_t kn[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) kn[r] = e + 1 + r < n ? s_keys[e + 1 + r] : ~0ull;
                uint32_t c = 0;
                bool go = true;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    go = go && e + 1 + r < n && (uint32_t)(kn[r] >> 40) == bi && kn[r] - ki < T;
                    c += go ? 1u : 0u;
                }
                if (c == 4)
                    for (uint32_t j = e + 5; j < n; ++j) {
                        const uint64_t kj = s_keys[j];
                        if ((uint32_t)(kj >> 40) != bi || kj - ki >= T) break;
                        ++c;
                    }
                s_cnt[e] = (uint16_t)c;
            }
            const uint32_t bfirst = g << (VXK_BUCKET_BITS - G);
            for (uint32_t bl = tid; bl < nbg; bl += BLOCK) {
                const uint32_t b = bfirst + bl;
                uint32_t a = 0, c = n;
                while (a < c) {
                    const uint32_t mid = (a + c) >> 1;
                    if ((uint32_t)(s_keys[mid] >> 40) < b) a = mid + 1; else c = mid;
                }
                offsets[b] = lo + a;
            }
            __syncthreads();
            // Canonical slots: thread t owns records [t * ITEMS, t * ITEMS + ITEMS).
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t e = tid * ITEMS + i;
                if (e < n) mine += s_cnt[e];
            }
        } else if (n <= fb_max) {
            // Slow path: the group's records, as a scratch copy when in place.
            if (!in.keys) {
                for (uint32_t e = tid; e < n; e += BLOCK) {
                    scr_keys[lo + e] = keys[lo + e];
                    scr_nonces[lo + e] = nonces[lo + e];
                }
                src_k = scr_keys + lo;
                src_n = scr_nonces + lo;
                __syncthreads();
            }
            slow_sort_group<BLOCK, CAPMAX>(src_k, src_n, n, keys, nonces, lo, g, G, offsets, s_keys, s_nonces);
            for (uint32_t e = tid; e < n; e += BLOCK) mine += pairs_after(keys + lo, e, n, T);
        } else {
            if (tid == 0) atomicOr(dev_status, (uint32_t)VXK_DEV_STATUS_GROUP_TOO_LARGE);
        }
        uint64_t ctot;
        const uint64_t my_off = vxd::block_exclusive_scan<BLOCK>(mine, s_wave, &ctot);
        // Publish this group's total at once, so that later groups can pass it
        // in their look-back while this one keeps working.
        if (tid == 0) lb_store(&words[g], kLbAgg | ctot);
        const uint64_t base = lookback<BLOCK>(words, g, spin_limit, dev_status, s_lb, s_wave);
        if (tid == 0) {
            lb_store(&words[g], kLbPrefix | (base + ctot));
            if (g == ngroups - 1) *t2_count = base + ctot;
        }
        if (fast && ctot) {
            // A group's pairs fit 32 bits (at most CAPMAX^2 / 2).  First slot of
            // each record, then the slots in windows of SLOTS (one window unless
            // the keys are crowded); counts are re-read from LDS per window,
            // which keeps the hash loop's live registers few.
            const uint32_t tot = (uint32_t)ctot, off = (uint32_t)my_off;
            {
                uint32_t r = off;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t e = tid * ITEMS + i;
                    if (e < n) {
                        s_first[e] = r;
                        r += s_cnt[e];
                    }
                }
            }
#pragma unroll 1
            for (uint32_t w0 = 0; w0 < tot; w0 += SLOTS) {
                const uint32_t w1 = min(w0 + (uint32_t)SLOTS, tot);
                uint32_t f = off;
#pragma unroll 1
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t e = tid * ITEMS + i;
                    const uint32_t c = e < n ? (uint32_t)s_cnt[e] : 0u;
                    const uint32_t a = max(f, w0), b = min(f + c, w1);
                    for (uint32_t q = a; q < b; ++q) s_slot[q - w0] = (uint16_t)e;
                    f += c;
                }
                __syncthreads();
                const uint32_t nq = w1 - w0;
                uint4 *out = t2 + base + w0;
                const uint64_t room = base + w0 < t2cap ? t2cap - (base + w0) : 0;
#pragma unroll 1
                for (uint32_t qr = tid; qr < nq; qr += BLOCK) {
                    const uint32_t e = s_slot[qr];
                    const uint32_t j = e + 1 + (w0 + qr - s_first[e]);
                    const uint32_t na = s_nonces[e], nb = s_nonces[j];
                    const uint64_t h = vxd::h2(key, na, nb);
                    if (qr < room) out[qr] = make_uint4(na, nb, (uint32_t)h, (uint32_t)(h >> 32));
                }
                __syncthreads();
            }
        } else if (!fast && ctot) {
            // Slow path: pairs in canonical order by one thread's sequential
            // walk (rare; correctness only).
            if (tid == 0) {
                uint64_t idx = base;
                for (uint32_t e = 0; e < n; ++e) {
                    const uint32_t c = pairs_after(keys + lo, e, n, T);
                    for (uint32_t q = 0; q < c; ++q) {
                        const uint32_t a = nonces[lo + e], b = nonces[lo + e + 1 + q];
                        const uint64_t h = vxd::h2(key, a, b);
                        if (idx < t2cap) t2[idx] = make_uint4(a, b, (uint32_t)h, (uint32_t)(h >> 32));
                        ++idx;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of u64 (pair counts -> Table-2 bases).
// ---------------------------------------------------------------------------

constexpr int kScanBlock = 1024;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanBlock * kScanPer;

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint64_t *__restrict__ in,
                                                           uint32_t n, uint64_t *__restrict__ part) {
    __shared__ uint64_t s_wave[kScanBlock / 64 + 1];
    const uint64_t t0 = (uint64_t)blockIdx.x * kScanTile;
    uint64_t sum = 0;
    for (int i = 0; i < kScanPer; ++i) {
        const uint64_t ix = t0 + (uint64_t)i * kScanBlock + threadIdx.x;
        if (ix < n) sum += in[ix];
    }
    sum = vxd::block_sum<kScanBlock>(sum, s_wave);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_partials(uint64_t *__restrict__ part,
                                                             uint32_t nparts,
                                                             uint64_t *__restrict__ total_out) {
    __shared__ uint64_t s[kScanTile];
    __shared__ uint64_t s_wave[kScanBlock / 64 + 1];
    for (uint32_t i = threadIdx.x; i < nparts; i += kScanBlock) s[i] = part[i];
    __syncthreads();
    const uint64_t total = vxd::lds_exclusive_scan<kScanBlock>(s, (int)nparts, s_wave);
    for (uint32_t i = threadIdx.x; i < nparts; i += kScanBlock) part[i] = s[i];
    if (threadIdx.x == 0 && total_out) *total_out = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint64_t *__restrict__ in, uint32_t n,
                                                          const uint64_t *__restrict__ part,
                                                          uint64_t *__restrict__ out) {
    __shared__ uint64_t s[kScanTile];
    __shared__ uint64_t s_wave[kScanBlock / 64 + 1];
    const uint64_t t0 = (uint64_t)blockIdx.x * kScanTile;
    const uint32_t m = (uint32_t)min((uint64_t)kScanTile, (uint64_t)n - t0);
    for (uint32_t i = threadIdx.x; i < m; i += kScanBlock) s[i] = in[t0 + i];
    __syncthreads();
    vxd::lds_exclusive_scan<kScanBlock>(s, (int)m, s_wave);
    const uint64_t base = part[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < m; i += kScanBlock) out[t0 + i] = base + s[i];
}

__global__ void k_zero_u64(uint64_t *__restrict__ p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_reset_words(uint32_t *__restrict__ p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

// Work-groups of `kernel` that are resident on the whole device at once:
// persistent kernels are launched with exactly this many, so none waits for
// a second round (a late round would leave most CUs idle at the tail).
static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return 256;
    return cus;
}

template <typename K>
static uint32_t resident_grid(K kernel, int block) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return (uint32_t)(cus * per_cu);
}

static TileGeom geom_chunks(uint64_t n, uint64_t chunk) {
    TileGeom g;
    g.mode = 0;
    g.q = 1;
    g.chunk = chunk;
    g.n = n;
    g.seg = nullptr;
    g.seg_end = nullptr;
    return g;
}

// seg_end == NULL: back-to-back segments (segment s ends at seg[s + 1]).
static TileGeom geom_segments(const uint32_t *seg, const uint32_t *seg_end, uint32_t q) {
    TileGeom g;
    g.mode = 1;
    g.q = q;
    g.chunk = 0;
    g.n = 0;
    g.seg = seg;
    g.seg_end = seg_end ? seg_end : seg + 1;
    return g;
}

constexpr int kHashBlock = 256;
constexpr int kHistBlock = 256;
constexpr int kColBlock = 1024;
constexpr int kSortBlock = 512;
constexpr int kFallbackBlock = 1024;
constexpr int kFallbackGrid = 256;

hipError_t launch_hash_filter(const uint32_t key_words[8], uint64_t n, uint32_t tiles, uint64_t chunk,
                              uint32_t pbits, uint32_t prefix, uint64_t *keys, uint32_t *nonces, uint64_t cap,
                              unsigned long long *count, hipStream_t s) {
    Key key;
    for (int i = 0; i < 8; ++i) key.w[i] = key_words[i];
    hipLaunchKernelGGL((k_hash_filter<kHashBlock, 8>), dim3(tiles), dim3(kHashBlock), 0, s, key, n, chunk, pbits,
                       prefix, keys, nonces, cap, count);
    return hipGetLastError();
}

uint32_t hash_scatter_grid(bool small) {
    static const uint32_t g = resident_grid(k_hash_scatter<kHashBlock, kHashScatterItems, kHashScatterMaxDigits>,
                                            kHashBlock);
    static const uint32_t g64 = resident_grid(k_hash_scatter<kHashBlock, kHashScatterItems, 64>, kHashBlock);
    return small ? g64 : g;
}

hipError_t launch_hash_scatter(const uint32_t key_words[8], uint64_t n, uint32_t bits, uint32_t R, uint64_t *keys,
                               uint32_t *nonces, uint32_t *fill, uint32_t *status, hipStream_t s) {
    if (bits < 1 || bits > (uint32_t)kHashScatterMaxBits) return hipErrorInvalidValue;
    Key key;
    for (int i = 0; i < 8; ++i) key.w[i] = key_words[i];
    constexpr uint64_t SUB = (uint64_t)kHashBlock * kHashScatterItems;
    const uint64_t nsub = (n + SUB - 1) / SUB;
    // Up to 64 digits (the first digit of three-pass plots, k >= 29, and of
    // small plots) the kernel's LDS and 80 VGPRs fit six work-groups per CU
    // instead of five.
    const bool small = bits <= 6;
    const uint32_t grid = hash_scatter_grid(small);
    const uint64_t per = (nsub + grid - 1) / grid;
    const uint32_t used = (uint32_t)((nsub + per - 1) / per);
    if (small)
        hipLaunchKernelGGL((k_hash_scatter<kHashBlock, kHashScatterItems, 64>), dim3(used),
                           dim3(kHashBlock), 0, s, key, n, per, bits, R, keys, nonces, fill, status);
    else
        hipLaunchKernelGGL((k_hash_scatter<kHashBlock, kHashScatterItems, kHashScatterMaxDigits>), dim3(used),
                           dim3(kHashBlock), 0, s, key, n, per, bits, R, keys, nonces, fill, status);
    return hipGetLastError();
}

hipError_t launch_hash_pass(const HashPassList &L, uint32_t *ticket, hipStream_t s) {
    static_assert(1 << kHashPassMaxBits <= kHashBlock, "one thread per digit");
    if (L.nh > (uint32_t)kHashPassMaxSlices || L.np > (uint32_t)kHashPassMaxSlices) return hipErrorInvalidValue;
    uint32_t bits = 1;
    for (uint32_t i = 0; i < L.nh; ++i) {
        if (L.h[i].bits < 1 || L.h[i].bits > (uint32_t)kHashPassMaxBits) return hipErrorInvalidValue;
        bits = max(bits, L.h[i].bits);
    }
    for (uint32_t i = 0; i < L.np; ++i) {
        if (L.p[i].bits < 1 || L.p[i].bits > (uint32_t)kHashPassMaxBits || L.p[i].per < 1 || L.p[i].shift < 32 ||
            L.p[i].shift + L.p[i].bits > 64)
            return hipErrorInvalidValue;  // digits lie in the key's high word
        bits = max(bits, L.p[i].bits);
    }
    const uint32_t sub = L.sub ? L.sub : kHashScatterSub;
    if (sub != kHashScatterSub && sub != kHashPassWideSub) return hipErrorInvalidValue;
    const uint64_t nt = (uint64_t)L.h_items + L.p_items;
    if (nt == 0) return hipSuccess;
    // Digits up to 7 bits take the kernel whose LDS fits six 256-thread (or
    // three 512-thread) work-groups on a CU; 8-bit digits the one with room
    // for 256 counters.  512-thread work-groups file sub-tiles of 4096
    // records, whose runs per digit are twice as long.
    constexpr int WB = 2 * kHashBlock;
    static const uint32_t grid7 = resident_grid(k_hash_pass<kHashBlock, kHashScatterItems, 128>, kHashBlock);
    static const uint32_t grid8 = resident_grid(k_hash_pass<kHashBlock, kHashScatterItems, 256>, kHashBlock);
    static const uint32_t gridw7 = resident_grid(k_hash_pass<WB, kHashScatterItems, 128>, WB);
    static const uint32_t gridw8 = resident_grid(k_hash_pass<WB, kHashScatterItems, 256>, WB);
    static_assert(WB * kHashScatterItems == (int)kHashPassWideSub, "wide sub-tile");
    const bool wide = sub == kHashPassWideSub;
    const uint32_t grid = wide ? (bits <= 7 ? gridw7 : gridw8) : (bits <= 7 ? grid7 : grid8);
    const uint32_t used = nt < grid ? (uint32_t)nt : grid;
    if (wide && bits <= 7)
        hipLaunchKernelGGL((k_hash_pass<WB, kHashScatterItems, 128>), dim3(used), dim3(WB), 0, s, L, ticket);
    else if (wide)
        hipLaunchKernelGGL((k_hash_pass<WB, kHashScatterItems, 256>), dim3(used), dim3(WB), 0, s, L, ticket);
    else if (bits <= 7)
        hipLaunchKernelGGL((k_hash_pass<kHashBlock, kHashScatterItems, 128>), dim3(used), dim3(kHashBlock), 0, s, L,
                           ticket);
    else
        hipLaunchKernelGGL((k_hash_pass<kHashBlock, kHashScatterItems, 256>), dim3(used), dim3(kHashBlock), 0, s, L,
                           ticket);
    return hipGetLastError();
}

hipError_t launch_region_scan_slices(const uint32_t *fill, uint32_t slices, uint32_t stride, uint32_t nd,
                                     uint32_t R, uint32_t *gstart, hipStream_t s) {
    hipLaunchKernelGGL(k_region_scan_slices<kColBlock>, dim3(1), dim3(kColBlock), 0, s, fill, slices, stride, nd,
                       R, gstart);
    return hipGetLastError();
}

hipError_t launch_region_scan(const uint32_t *fill, uint32_t nd, uint32_t R, uint32_t *seg_lo, uint32_t *seg_hi,
                              uint32_t *gstart, hipStream_t s) {
    hipLaunchKernelGGL(k_region_scan<kColBlock>, dim3(1), dim3(kColBlock), 0, s, fill, nd, R, seg_lo, seg_hi,
                       gstart);
    return hipGetLastError();
}

struct Words16 {
    uint32_t w[16];
};

__global__ void k_put_words(uint32_t *__restrict__ p, Words16 v, uint32_t n) {
    if (threadIdx.x < n) p[threadIdx.x] = v.w[threadIdx.x];
}

hipError_t launch_put_words(uint32_t *p, const uint32_t *values, uint32_t n, hipStream_t s) {
    if (n > 16) return hipErrorInvalidValue;
    Words16 v = {};
    for (uint32_t i = 0; i < n; ++i) v.w[i] = values[i];
    hipLaunchKernelGGL(k_put_words, dim3(1), dim3(64), 0, s, p, v, n);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_reset(uint32_t *words, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_words, dim3(1), dim3(256), 0, s, words, n);
    return hipGetLastError();
}

hipError_t launch_hash_table1(const uint32_t key_words[8], uint64_t n, uint32_t tiles, uint64_t chunk,
                              uint64_t *keys, uint32_t *hist, uint32_t hist_bits, hipStream_t s) {
    Key key;
    for (int i = 0; i < 8; ++i) key.w[i] = key_words[i];
    hipLaunchKernelGGL(k_hash_table1<kHashBlock>, dim3(tiles), dim3(kHashBlock), 0, s, key, n, chunk,
                       keys, hist, hist_bits);
    return hipGetLastError();
}

hipError_t launch_hist_chunks(const uint64_t *keys, uint64_t n, uint32_t tiles, uint64_t chunk,
                              uint32_t shift, uint32_t bits, uint32_t *hist, hipStream_t s) {
    hipLaunchKernelGGL(k_digit_hist<kHistBlock>, dim3(tiles), dim3(kHistBlock), 0, s, keys,
                       geom_chunks(n, chunk), shift, bits, hist);
    return hipGetLastError();
}

hipError_t launch_hist_segments(const uint64_t *keys, const uint32_t *seg, const uint32_t *seg_end, uint32_t nseg,
                                uint32_t q, uint32_t shift, uint32_t bits, uint32_t *hist, hipStream_t s) {
    hipLaunchKernelGGL(k_digit_hist<kHistBlock>, dim3(nseg * q), dim3(kHistBlock), 0, s, keys,
                       geom_segments(seg, seg_end, q), shift, bits, hist);
    return hipGetLastError();
}

hipError_t launch_colscan(const uint32_t *hist, uint32_t *off, uint32_t nseg, uint32_t rps,
                          uint32_t ncol, const uint32_t *seg_base, uint32_t *gstart, uint32_t n_groups,
                          uint32_t n_total, hipStream_t s) {
    hipLaunchKernelGGL(k_colscan<kColBlock>, dim3(nseg), dim3(kColBlock), 0, s, hist, off, rps, ncol,
                       seg_base, gstart, n_groups, n_total);
    return hipGetLastError();
}

// Digits of 7 to 9 bits use 8192-record sub-tiles (16+ records per digit run,
// one 1024-thread work-group per CU); narrower digits use 4096-record
// sub-tiles with several work-groups per CU; wider ones (tunings only) the
// big tile with room for 2048 digits.
template <typename... A>
static hipError_t launch_scatter_cfg(uint32_t bits, uint32_t grid, hipStream_t s, A... args) {
    if (bits <= 6)
        hipLaunchKernelGGL((k_scatter<512, 8, 64, false>), dim3(grid), dim3(512), 0, s, args..., Claim{});
    else if (bits <= 9)
        hipLaunchKernelGGL((k_scatter<1024, 8, 512, false>), dim3(grid), dim3(1024), 0, s, args..., Claim{});
    else
        hipLaunchKernelGGL((k_scatter<1024, 8, kMaxDigits, false>), dim3(grid), dim3(1024), 0, s, args...,
                           Claim{});
    return hipGetLastError();
}

hipError_t launch_scatter_chunks(const uint64_t *in_keys, const uint32_t *in_nonces,
                                 uint64_t *out_keys, uint32_t *out_nonces, const uint32_t *off,
                                 uint64_t n, uint32_t tiles, uint64_t chunk, uint32_t shift,
                                 uint32_t bits, hipStream_t s) {
    return launch_scatter_cfg(bits, tiles, s, in_keys, in_nonces, out_keys, out_nonces, off,
                              geom_chunks(n, chunk), shift, bits);
}

hipError_t launch_scatter_segments(const uint64_t *in_keys, const uint32_t *in_nonces,
                                   uint64_t *out_keys, uint32_t *out_nonces, const uint32_t *off,
                                   const uint32_t *seg, const uint32_t *seg_end, uint32_t nseg, uint32_t q,
                                   uint32_t shift, uint32_t bits, hipStream_t s) {
    return launch_scatter_cfg(bits, nseg * q, s, in_keys, in_nonces, out_keys, out_nonces, off,
                              geom_segments(seg, seg_end, q), shift, bits);
}

hipError_t launch_scatter_claim(const uint64_t *in_keys, const uint32_t *in_nonces, uint64_t *out_keys,
                                uint32_t *out_nonces, const uint32_t *seg, const uint32_t *seg_end, uint32_t nseg,
                                uint32_t q, uint32_t shift, uint32_t bits, uint32_t *fill, uint32_t R,
                                uint32_t *status, hipStream_t s) {
    if (bits < 1 || bits > (uint32_t)kClaimMaxBits) return hipErrorInvalidValue;
    const Claim c{fill, R, status};
    const TileGeom g = geom_segments(seg, seg_end, q);
    if (bits <= 6)
        hipLaunchKernelGGL((k_scatter<512, 8, 64, true>), dim3(nseg * q), dim3(512), 0, s, in_keys, in_nonces,
                           out_keys, out_nonces, nullptr, g, shift, bits, c);
    else
        // 12288-record sub-tiles (148 KB of LDS, one work-group per CU):
        // runs of about 96 records per 7-bit digit, which write faster than
        // the 64 of 8192-record sub-tiles (k=31: 23.6 against 24.6 ms for
        // two passes), while 4096-record sub-tiles at twice the occupancy
        // were slower still (28.4 ms).
        hipLaunchKernelGGL((k_scatter<1024, 12, 512, true>), dim3(nseg * q), dim3(1024), 0, s, in_keys, in_nonces,
                           out_keys, out_nonces, nullptr, g, shift, bits, c);
    return hipGetLastError();
}

hipError_t launch_region_bounds(uint32_t *fill, uint32_t r0, uint32_t nregions, uint32_t R, uint32_t *seg_lo,
                                uint32_t *seg_hi, hipStream_t s) {
    const uint32_t blocks = (nregions + 255) / 256;
    hipLaunchKernelGGL(k_region_bounds, dim3(blocks < 1024 ? blocks : 1024), dim3(256), 0, s, fill, r0, nregions,
                       R, seg_lo, seg_hi);
    return hipGetLastError();
}

hipError_t launch_groupsort(uint64_t *keys, uint32_t *nonces, const uint64_t *in_keys, const uint32_t *in_nonces,
                            const uint32_t *in_lo, const uint32_t *in_hi, const uint32_t *gstart, uint32_t G, uint32_t cap,
                            uint32_t *offsets, uint32_t n_total, uint32_t *ovf_count, uint32_t *ovf_list, uint64_t T,
                            uint8_t *pcnt, uint32_t g0, uint32_t gcount, uint32_t *ticket, uint64_t *csum, uint32_t cb,
                            hipStream_t s) {
    // Group capacities up to kGroupCapFast take the kernel that fits four
    // work-groups on a CU; larger ones the 3072-record kernel (three).
    static const uint32_t resident_fast = resident_grid(k_groupsort<kSortBlock, kGroupCapFast>, kSortBlock);
    static const uint32_t resident_max = resident_grid(k_groupsort<kSortBlock, kGroupCapMax>, kSortBlock);
    const bool fast = cap <= (uint32_t)kGroupCapFast;
    const uint32_t grid = min(gcount, fast ? resident_fast : resident_max);
    if (grid == 0) return hipSuccess;
    const SortArgs A{keys, nonces, GroupIn{in_keys, in_nonces, in_lo, in_hi}, gstart, offsets, ovf_count, ovf_list,
                     pcnt, reinterpret_cast<unsigned long long *>(csum), T, G, cap, n_total, cb};
    if (fast)
        hipLaunchKernelGGL((k_groupsort<kSortBlock, kGroupCapFast>), dim3(grid), dim3(kSortBlock), 0, s, A, g0,
                           gcount, ticket);
    else
        hipLaunchKernelGGL((k_groupsort<kSortBlock, kGroupCapMax>), dim3(grid), dim3(kSortBlock), 0, s, A, g0,
                           gcount, ticket);
    return hipGetLastError();
}

hipError_t launch_group_fallback(uint64_t *keys, uint32_t *nonces, const uint64_t *in_keys,
                                 const uint32_t *in_nonces, const uint32_t *in_lo, const uint32_t *in_hi,
                                 uint64_t *scr_keys,
                                 uint32_t *scr_nonces, const uint32_t *gstart, uint32_t G,
                                 uint32_t *offsets, const uint32_t *ovf_count, const uint32_t *ovf_list,
                                 uint32_t *status, uint64_t T, uint8_t *pcnt, uint64_t *csum, uint32_t cb,
                                 hipStream_t s) {
    const GroupIn in{in_keys, in_nonces, in_lo, in_hi};
    hipLaunchKernelGGL(k_group_fallback<kFallbackBlock>, dim3(kFallbackGrid), dim3(kFallbackBlock), 0,
                       s, keys, nonces, in, scr_keys, scr_nonces, gstart, G, offsets, ovf_count, ovf_list,
                       (uint32_t)kFallbackMax, status, T, pcnt, reinterpret_cast<unsigned long long *>(csum), cb);
    return hipGetLastError();
}

hipError_t launch_match_count(const uint64_t *keys, uint32_t n_total, uint32_t chunk_bits, uint64_t T,
                              uint64_t *counts, uint8_t *pcnt, hipStream_t s) {
    const uint32_t nchunks = (n_total + (1u << chunk_bits) - 1) >> chunk_bits;
    static const uint32_t resident = resident_grid(k_match_count<kMatchBlock, kMatchCap>, kMatchBlock);
    const uint32_t grid = min(nchunks, resident);
    hipLaunchKernelGGL((k_match_count<kMatchBlock, kMatchCap>), dim3(grid), dim3(kMatchBlock), 0, s,
                       keys, n_total, chunk_bits, T, counts, pcnt);
    return hipGetLastError();
}

hipError_t launch_scan_u64(const uint64_t *in, uint32_t n, uint64_t *out, uint64_t *part,
                           uint64_t *total, hipStream_t s) {
    const uint32_t nparts = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(kScanBlock), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanBlock), 0, s, part, nparts, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(nparts), dim3(kScanBlock), 0, s, in, n, part, out);
    return hipGetLastError();
}

uint32_t scan_parts(uint32_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_chunk_sums(const uint8_t *pcnt, const uint64_t *keys, uint32_t n_total, uint32_t chunk_bits,
                             uint64_t T, uint64_t *counts, const uint32_t *r_lo, const uint32_t *r_hi,
                             uint32_t last, uint32_t max_chunks, hipStream_t s) {
    constexpr int kBlock = 256;
    const uint32_t grid = max(1u, min((max_chunks + kBlock / 64 - 1) / (kBlock / 64), 8192u));
    hipLaunchKernelGGL(k_chunk_sums<kBlock>, dim3(grid), dim3(kBlock), 0, s, pcnt, keys, n_total, chunk_bits, T,
                       counts, r_lo, r_hi, last);
    return hipGetLastError();
}

hipError_t launch_scan_range(const uint64_t *counts, uint64_t *bases, uint32_t n_total, uint32_t chunk_bits,
                             const uint32_t *r_lo, const uint32_t *r_hi, uint32_t last, uint64_t *acc,
                             uint64_t *t2_count, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_range<1024>, dim3(1), dim3(1024), 0, s, counts, bases, n_total, chunk_bits, r_lo,
                       r_hi, last, acc, t2_count);
    return hipGetLastError();
}

hipError_t launch_match_emit(const uint32_t key_words[8], const uint64_t *keys, const uint32_t *nonces,
                             const uint8_t *pcnt, uint32_t n_total, uint32_t chunk_bits, uint64_t T,
                             const uint64_t *chunk_base, void *t2, uint64_t cap, const uint32_t *r_lo,
                             const uint32_t *r_hi, uint32_t last, uint32_t max_chunks, uint32_t wg_per_cu,
                             uint32_t *ticket, hipStream_t s) {
    Key key;
    for (int i = 0; i < 8; ++i) key.w[i] = key_words[i];
    static const uint32_t resident = resident_grid(k_match_emit<kMatchBlock, kMatchCap, kMatchSlots>, kMatchBlock);
    static const uint32_t per_cu = max(1u, resident / max(1u, (uint32_t)device_cus()));
    const uint32_t want = wg_per_cu ? min(wg_per_cu, per_cu) * (uint32_t)device_cus() : resident;
    const uint32_t grid = max(1u, min(max_chunks, want));
    MatchArgs A{{}, keys, nonces, pcnt, chunk_base, (uint4 *)t2, cap, T, n_total, chunk_bits};
    for (int i = 0; i < 8; ++i) A.key[i] = key_words[i];
    hipLaunchKernelGGL((k_match_emit<kMatchBlock, kMatchCap, kMatchSlots>), dim3(grid), dim3(kMatchBlock),
                       0, s, A, r_lo, r_hi, last, ticket);
    return hipGetLastError();
}

__global__ void k_store_list(PipeList L, PipeList *dst) {
    if (threadIdx.x == 0) *dst = L;
}

hipError_t launch_pipe(const PipeList &L, PipeList *d_list, uint32_t *ticket, hipStream_t s) {
    for (int r = 0; r < 4; ++r)
        if (L.n[r] > (uint32_t)kPipeMaxLists) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < L.n[0]; ++i)
        if (L.h[i].bits < 1 || L.h[i].bits > (uint32_t)kPipeMaxBits) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < L.n[1]; ++i)
        if (L.p[i].bits < 1 || L.p[i].bits > (uint32_t)kPipeMaxBits || L.p[i].per < 1 || L.p[i].shift < 32 ||
            L.p[i].shift + L.p[i].bits > 64)
            return hipErrorInvalidValue;  // digits lie in the key's high word
    const uint64_t nt = (uint64_t)L.items[0] + L.items[1] + L.items[2] + L.items[3];
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_store_list, dim3(1), dim3(64), 0, s, L, d_list);
    static const uint32_t grid = resident_grid(k_pipe<kPipeBlock>, kPipeBlock);
    const uint32_t used = nt < grid ? (uint32_t)nt : grid;
    hipLaunchKernelGGL(k_pipe<kPipeBlock>, dim3(used), dim3(kPipeBlock), 0, s, (const PipeList *)d_list, ticket);
    return hipGetLastError();
}

hipError_t launch_group_match(const uint32_t key_words[8], uint64_t *keys, uint32_t *nonces, const uint64_t *in_keys,
                              const uint32_t *in_nonces, const uint32_t *in_lo, const uint32_t *in_hi,
                              uint64_t *scr_keys, uint32_t *scr_nonces, const uint32_t *gstart, uint32_t G,
                              uint32_t cap, uint32_t *offsets, uint32_t n_total, uint64_t T, uint32_t *ticket,
                              uint64_t *words, uint32_t *dev_status, void *t2, uint64_t t2cap, uint64_t *t2_count,
                              uint32_t spin_limit, hipStream_t s) {
    Key key;
    for (int i = 0; i < 8; ++i) key.w[i] = key_words[i];
    const GroupIn in{in_keys, in_nonces, in_lo, in_hi};
    // Group capacities up to kGroupCapFast take the kernel that fits four
    // work-groups on a CU; larger ones the 3072-record kernel.
    static const uint32_t resident_fast =
        resident_grid(k_group_match<kSortBlock, kGroupCapFast, kMatchSlots>, kSortBlock);
    static const uint32_t resident_max =
        resident_grid(k_group_match<kSortBlock, kGroupCapMax, kMatchSlots>, kSortBlock);
    const bool fast = cap <= (uint32_t)kGroupCapFast;
    const uint32_t grid = min(1u << G, fast ? resident_fast : resident_max);
    if (fast)
        hipLaunchKernelGGL((k_group_match<kSortBlock, kGroupCapFast, kMatchSlots>), dim3(grid), dim3(kSortBlock), 0,
                           s, key, keys, nonces, in, scr_keys, scr_nonces, gstart, G, cap, offsets, n_total, T,
                           ticket, words, dev_status, (uint4 *)t2, t2cap, t2_count, spin_limit,
                           (uint32_t)kFallbackMax);
    else
        hipLaunchKernelGGL((k_group_match<kSortBlock, kGroupCapMax, kMatchSlots>), dim3(grid), dim3(kSortBlock), 0,
                           s, key, keys, nonces, in, scr_keys, scr_nonces, gstart, G, cap, offsets, n_total, T,
                           ticket, words, dev_status, (uint4 *)t2, t2cap, t2_count, spin_limit,
                           (uint32_t)kFallbackMax);
    return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t *p, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(min((n + 1023) / 1024, 4096u)), dim3(1024), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace vxk
