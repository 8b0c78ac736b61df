// C ABI of libvx (declared in include/vx.h): argument checks, the per-plot
// plan (partition digits, group sizes, tile counts), the workspace layout,
// and the launch sequence of each call.  No call allocates device memory.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "errors.h"
#include "kernels.h"
#include "vx.h"

namespace {

thread_local char g_err[512] = "";

vx_status fail(vx_status st, const char *msg) {
    snprintf(g_err, sizeof(g_err), "%s", msg);
    return st;
}

vx_status fail_hip(hipError_t e, const char *where) {
    snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
    return VX_ERR_DEVICE;
}

#define VX_HIP(call, where)                              \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return fail_hip(e_, where); \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// How one plot is cut into kernels.  Every field only moves work around;
// outputs never depend on it.
constexpr int kMaxPasses = 3;
constexpr uint32_t kMaxSlices = 16;
// Measured at k=31: the two streams barely overlap (the match's and the
// partition's work-groups do not share CUs in practice), and the pipelined
// plot was slower than the sequential one, so pipelining is opt-in.
constexpr uint32_t kDefaultSlices = 1;
// A plot hashed in slices files each slice's records by the second digit
// beside the next slice's hash (run_sliced_front).
constexpr uint32_t kMaxHashSlices = 32;
// Each hash slice's first-pass fill counters start on a 256-byte line of
// their own: a slice's hash claims room with atomics on them while the next
// launch reads them, and two slices sharing a line (16 counters at k = 29)
// made every other launch of a k=29 plot twice as slow.
inline uint32_t slice_fill_stride(uint32_t d0) { return ((1u << d0) + 63u) & ~63u; }
// Measured (one box, median plot time, 1 / 4 / 16 slices, the second pass
// in the hash launches): k=31 114.0 / 108.8 / 103.8 ms, k=30 57.8 / 55.0 /
// 53.4, k=29 29.2 / 27.5 / 26.9, k=27 6.63 / 6.26 / 6.37, k=26 3.25 / 3.13 /
// 3.43, k=25 1.73 / 1.62 / 2.06; below k=25 the hash is too short to hide a
// pass.  At k=28 the sliced split needs a third pass, which pays once the
// launches also file it (16 slices: 13.2 against 13.65 ms in one launch).
uint32_t default_hash_slices(uint32_t k) { return k >= 28 ? 16 : (k >= 25 ? 4 : 1); }
// A plot's work after its first two partition passes can be pipelined over
// slices (run_pipe_tail).
constexpr uint32_t kMaxTailSlices = 16;
uint32_t default_tail_slices(uint32_t /*k*/) { return 1; }

struct Plan {
    uint32_t k = 0;
    uint64_t n = 0;          // 2^k records
    uint32_t key_words[8] = {};
    uint64_t T = 0;
    uint32_t G = 0;          // sort groups = 2^G leading-bit prefixes
    uint32_t npass = 0;      // MSD partition passes over those G bits
    uint32_t D[kMaxPasses] = {};   // digit bits per pass
    uint32_t pre[kMaxPasses] = {}; // bits consumed before each pass
    uint32_t Q[kMaxPasses] = {};   // tiles per input segment (passes >= 1)
    uint32_t W = 0;          // tiles of hash + pass 0
    uint64_t chunk1 = 0;     // records per pass-0 tile
    uint32_t cap = 0;        // LDS capacity of a sort group
    uint32_t cb = 0;         // match chunk = 2^cb consecutive Table-1 records
    bool fused = false;      // plot: one fused sort + match kernel instead of two
    uint32_t slices = 1;     // plot: pipeline slices of the passes after the first (1 = none)
    bool hs = false;         // plot: region passes (the hash does the first; see make_plan)
    uint32_t R[kMaxPasses] = {};  // hs: records per region of each pass (pass 0: per hash slice)
    uint32_t hq = 1;         // plot: nonce slices of the hash (>= 2: see run_sliced_front)
    uint32_t zt = 1;         // plot: slices of the pipelined tail (>= 2: see run_pipe_tail)
    bool deep = false;       // plot: the sliced hash launches file all three passes (run_sliced_front)
    uint32_t hsub = vxk::kHashScatterSub;  // plot: records per item of the sliced hash's launches
    int staged = -1;         // >= 0: one chunk (of 2^staged) of a staged plot; see vx_stage_plot
};

uint32_t clampu(int64_t v, int64_t lo, int64_t hi) {
    return (uint32_t)(v < lo ? lo : (v > hi ? hi : v));
}

vx_status check_params(const vx_plot_params *p, uint32_t max_k = 31) {
    if (!p) return fail(VX_ERR_INVALID_ARG, "params is NULL");
    if (p->k < 1 || p->k > max_k)
        return fail(VX_ERR_INVALID_ARG, max_k == 31 ? "k must be in [1, 31] (k = 32: the chunk calls)"
                                                    : "k must be in [1, 32]");
    if (p->bucket_bits != VX_BUCKET_BITS) return fail(VX_ERR_INVALID_ARG, "bucket_bits must be 24");
    return VX_OK;
}

// records: the table's size when it is not 2^k (a chunk of a chunked plot,
// at most 2^32 - 1); 0 = 2^k.  Groups, digits and the threshold follow k.
// staged >= 0: the plan of a staged plot (records = 0) or of one of its
// 2^staged chunks (records = the chunk's), with region passes throughout.
vx_status make_plan(const vx_plot_params *p, const vx_tuning *t, Plan *pl, uint64_t records = 0,
                    uint32_t max_k = 31, int staged = -1) {
    vx_status st = check_params(p, max_k);
    if (st != VX_OK) return st;
    Plan P;
    P.k = p->k;
    P.n = records ? records : 1ull << p->k;
    for (int i = 0; i < 8; ++i)
        P.key_words[i] = (uint32_t)p->key[4 * i] | ((uint32_t)p->key[4 * i + 1] << 8) |
                         ((uint32_t)p->key[4 * i + 2] << 16) | ((uint32_t)p->key[4 * i + 3] << 24);
    P.T = p->match_threshold;
    vx_tuning z;
    memset(&z, 0, sizeof(z));
    if (!t) t = &z;
    // Sort groups of about 2048 records (half the LDS capacity).
    P.G = t->group_bits ? t->group_bits : clampu((int64_t)p->k - 11, 1, 21);
    if (P.G < 1 || P.G > 24) return fail(VX_ERR_UNSUPPORTED, "group_bits must be in [1, 24]");
    // A staged plot needs two passes (the stage holds the first), so small
    // staged plots take smaller groups.
    if (staged >= 0 && !t->group_bits && P.G < 10) P.G = 10;
    // Split G into passes of at most 9 bits so that every digit's run per
    // sub-tile spans whole cache lines.  The first pass scatters over the
    // whole table, where short runs cost the most, so it takes no more than
    // 7 bits once three passes are needed (7-7-6 at k=31).  When the hash
    // kernel does the first pass (see below), that digit stays at 8 bits or
    // less, and at most 6 with three passes: it files sub-tiles of only
    // 2048 records, so narrower digits keep its runs longer (measured at
    // k=28 and k=31).  With three passes up to G = 20 both later digits take
    // 7 bits, the width the claiming scatter writes fastest, and the hash the
    // rest: 4-7-7 at k=29, 5-7-7 at k=30, 6-7-7 at k=31 (6-6-6 and 6-7-6
    // were 0.4 and 0.5 ms slower at k=29 and k=30; 5-7-8 and 5-8-7 1.2 ms
    // slower at k=31).
    //
    // A pipelined plot (see run_pipelined; opt-in) instead keeps the later
    // passes at 6 bits, whose scatter fits on a CU next to two match
    // work-groups: 8-6-6 at k=31.
    if (t->pipeline_slices > kMaxSlices) return fail(VX_ERR_UNSUPPORTED, "pipeline_slices must be at most 16");
    if (t->region_pct > 1000) return fail(VX_ERR_UNSUPPORTED, "region_pct must be at most 1000");
    P.fused = t->fused_sort_match != 0;
    P.slices = t->pipeline_slices ? t->pipeline_slices : kDefaultSlices;
    if (P.fused) P.slices = 1;
    P.staged = staged;
    if (staged >= 0) {
        if (P.fused || t->separate_hash)
            return fail(VX_ERR_UNSUPPORTED, "staged plots use the fused hash and the split sort and match");
        P.slices = 1;
    }
    const bool hs_ok = (!records || staged >= 0) && !t->separate_hash;
    if (t->hash_slices > kMaxHashSlices) return fail(VX_ERR_UNSUPPORTED, "hash_slices must be at most 32");
    if (t->tail_slices > kMaxTailSlices) return fail(VX_ERR_UNSUPPORTED, "tail_slices must be at most 16");
    if (t->front_passes == 1 || t->front_passes > 3)
        return fail(VX_ERR_UNSUPPORTED, "front_passes must be 0, 2 or 3");
    if (t->front_subtile && t->front_subtile != vxk::kHashScatterSub && t->front_subtile != vxk::kHashPassWideSub)
        return fail(VX_ERR_UNSUPPORTED, "front_subtile must be 0, 2048 or 4096");

    // Hash slices: whole plots whose first two digits fit the sliced
    // kernel's 8 bits; the pipelined tail keeps its own split.
    // A staged plot (the stage and its chunks share one plan of the digits)
    // hashes in slices only if its launches file all three passes, and with
    // at most 4 chunks (a launch holds one third-pass descriptor per chunk).
    uint32_t hq = t->hash_slices ? t->hash_slices : default_hash_slices(P.k);
    if ((records && staged < 0) || staged > 2 || t->separate_hash || P.slices > 1 || P.G < 2 ||
        P.G > 2u * vxk::kHashPassMaxBits + (uint32_t)vxk::kHashPassMaxBits)
        hq = 1;
    // The digits of the passes for hq hash slices (see below).
    auto split = [&](uint32_t q, uint32_t &d0, uint32_t &d1, uint32_t &d2) -> vx_status {
        if (q > 1) {
            // Both digits of the sliced kernel take at most 8 bits.  Up to 16
            // group bits they are the only passes; above, the second and the
            // third (a claiming scatter of its own) take 7 bits, the width
            // those scatters write fastest, and the hash the rest.
            if (P.G <= 2u * vxk::kHashPassMaxBits) {
                d0 = (P.G + 1) / 2; d1 = P.G - d0; d2 = 0;
            } else {
                d1 = 7;
                d2 = std::min<uint32_t>(7, P.G - d1 - 1);
                d0 = P.G - d1 - d2;
            }
        } else if (P.G <= 9) {
            d0 = P.G; d1 = 0; d2 = 0;
        } else if (P.slices > 1 && P.G >= 13) {
            d0 = P.G - 12; d1 = 6; d2 = 6;
        } else if (hs_ok && P.G <= 13) {
            // The hash kernel files its first digit behind the ALU-bound
            // hash, so small plots give it 8 bits and the claiming scatter
            // the rest (autotuned: k=22 0.27 against 0.33 ms with 6-5, k=23
            // 0.44 against 0.48 ms with 6-6).
            d0 = std::min(8u, P.G - 1); d1 = P.G - d0; d2 = 0;
        } else if (P.G <= 17) {
            d0 = (P.G + 1) / 2;
            if (hs_ok) d0 = std::min(d0, 8u);
            d1 = P.G - d0; d2 = 0;
        } else if (hs_ok && P.G <= 20) {
            d0 = P.G - 14; d1 = 7; d2 = 7;
        } else {
            d0 = hs_ok ? 6 : 7; d1 = (P.G - d0 + 1) / 2; d2 = P.G - d0 - d1;
        }
        if (t->pass1_bits || t->pass2_bits) {
            d0 = t->pass1_bits ? t->pass1_bits : d0;
            if (d0 > P.G) return fail(VX_ERR_UNSUPPORTED, "pass1_bits must be at most group_bits");
            const uint32_t rest = P.G - d0;
            if (t->pass2_bits)
                d1 = t->pass2_bits;
            else if (q > 1)
                d1 = std::min<uint32_t>(rest, vxk::kHashPassMaxBits);
            else
                d1 = rest <= (uint32_t)vxk::kMaxDigitBits ? rest : (rest + 1) / 2;
            if (d1 > rest) return fail(VX_ERR_UNSUPPORTED, "pass1_bits + pass2_bits must be at most group_bits");
            d2 = rest - d1;
        }
        return VX_OK;
    };
    uint32_t d0, d1, d2;
    st = split(hq, d0, d1, d2);
    if (st != VX_OK) return st;
    if (hq > 1 && (!hs_ok || d0 > (uint32_t)vxk::kHashPassMaxBits || d1 == 0 ||
                   d1 > (uint32_t)vxk::kHashPassMaxBits || ((staged >= 0 ? 1ull << P.k : P.n) >> d0) < hq)) {
        hq = 1;  // beyond the sliced kernel: the plot hashes in one launch
        st = split(hq, d0, d1, d2);
        if (st != VX_OK) return st;
    }
    const uint32_t ds[kMaxPasses] = {d0, d1, d2};
    P.npass = 0;
    uint32_t used = 0;
    for (int i = 0; i < kMaxPasses; ++i) {
        if (ds[i] == 0) {
            if (i == 0) return fail(VX_ERR_UNSUPPORTED, "pass1_bits must be at least 1");
            continue;
        }
        if (ds[i] > (uint32_t)vxk::kMaxDigitBits)
            return fail(VX_ERR_UNSUPPORTED, "a partition pass may take at most 11 bits");
        P.D[P.npass] = ds[i];
        P.pre[P.npass] = used;
        used += ds[i];
        P.npass++;
    }
    P.W = t->h1_tiles ? t->h1_tiles : clampu((int64_t)(P.n >> 14), 1, 2048);
    if (P.W < 1 || P.W > 65536) return fail(VX_ERR_UNSUPPORTED, "h1_tiles must be in [1, 65536]");
    P.chunk1 = (P.n + P.W - 1) / P.W;
    // Segments of pass i hold 2^(k - pre) records on average (also in a
    // chunk, whose other segments are empty).
    const uint64_t dens = 1ull << P.k;
    for (uint32_t i = 1; i < P.npass; ++i)  // about 2^16 records per tile
        P.Q[i] = clampu((int64_t)((dens >> P.pre[i]) >> 16), 1, 256);
    // The split sort defaults to the capacity whose kernel fits four
    // work-groups on a CU.  With the default group bits a group holds 2048
    // records or fewer on average, and 2560 is 11 standard deviations above
    // 2048; larger groups take the fallback.
    P.cap = t->group_cap ? t->group_cap : (uint32_t)vxk::kGroupCapFast;
    if (P.cap < 64 || P.cap > (uint32_t)vxk::kGroupCapMax)
        return fail(VX_ERR_UNSUPPORTED, "group_cap must be in [64, 3072]");
    P.cb = t->match_chunk_bits ? t->match_chunk_bits : (uint32_t)vxk::kMatchChunkBitsMax;
    if (P.cb < 6 || P.cb > (uint32_t)vxk::kMatchChunkBitsMax)
        return fail(VX_ERR_UNSUPPORTED, "match_chunk_bits must be in [6, 11]");
    // Slices cut the first pass's segments; a plot with one pass has none.
    if (P.npass < 2) P.slices = 1;
    P.slices = std::min(P.slices, 1u << P.D[0]);
    if (P.slices < 1) P.slices = 1;
    // Plots with two or more passes fuse the first into the hash kernel,
    // and every pass files records into fixed-size regions, one per (input
    // segment, digit), claiming room with a global atomic per sub-tile run
    // (no histogram passes); the group sort then gathers each group from its
    // region into Table 1.  A region holds the expected records plus 8
    // standard deviations and some slack (fewer than one plot in 10^9
    // overflows one, which the device status reports).
    //
    // A pipelined plan with three passes keeps the contiguous passes: there a
    // slice's last pass would file into the buffer that still holds the
    // first pass's regions of later slices.
    P.hs = hs_ok && P.npass >= 2 && P.D[0] <= (uint32_t)vxk::kHashScatterMaxBits &&
           !(P.slices > 1 && P.npass > 2);
    for (uint32_t i = 1; i < P.npass; ++i)
        if (P.D[i] > (uint32_t)vxk::kClaimMaxBits) P.hs = false;
    // A chunk of a staged plot addresses only its own 2^-staged share of
    // each pass's regions.
    const uint32_t cbits = staged > 0 ? (uint32_t)staged : 0;
    for (uint32_t i = 0; P.hs && i < P.npass; ++i) {
        const uint32_t bits = P.pre[i] + P.D[i];
        const double mean = (double)((dens + (1ull << bits) - 1) >> bits);
        const uint32_t slack = i == 0 ? vxk::kHashScatterSub : 64u;
        P.R[i] = (uint32_t)(mean + 8.0 * std::sqrt(mean)) + slack;
        if (t->region_pct) P.R[i] = std::max<uint32_t>(1, (uint32_t)((uint64_t)P.R[i] * t->region_pct / 100));
        if (bits < cbits || ((uint64_t)P.R[i] << (bits - cbits)) >= (1ull << 32)) P.hs = false;
    }
    // Hash slices need the region passes, two or more passes, and both
    // leading digits within the sliced kernel's width; otherwise the plot
    // hashes in one launch.  Slice s hashes nonces [s * n / hq, (s + 1) * n /
    // hq) into 2^D[0] regions of its own, of R[0] records each.
    // A staged plan's slices cut the whole plot's 2^k nonces (a chunk's plan
    // has the chunk's record count in P.n), and its first-pass regions live
    // two slices at a time (see ring_slot).
    const uint64_t front_n = staged >= 0 ? dens : P.n;
    if (hq > 1 && P.hs && P.npass >= 2 && P.D[0] <= (uint32_t)vxk::kHashPassMaxBits &&
        P.D[1] <= (uint32_t)vxk::kHashPassMaxBits && (front_n >> P.D[0]) >= hq) {
        const double mean = (double)(((front_n + hq - 1) / hq + (1ull << P.D[0]) - 1) >> P.D[0]);
        uint32_t r0 = (uint32_t)(mean + 8.0 * std::sqrt(mean)) + vxk::kHashScatterSub;
        if (t->region_pct) r0 = std::max<uint32_t>(1, (uint32_t)((uint64_t)r0 * t->region_pct / 100));
        if (((uint64_t)r0 * (staged >= 0 ? 1 : hq) << P.D[0]) < (1ull << 32)) {
            P.hq = hq;
            P.R[0] = r0;
        }
    }
    // The pipelined tail: whole plots with region passes, the split sort (of
    // the 2560-record kernel) and match, and a third digit (if any) within
    // the filing kernel's 7 bits; slices cut the second pass's regions.
    {
        const uint32_t zt = t->tail_slices ? t->tail_slices : default_tail_slices(P.k);
        if (zt > 1 && !records && staged < 0 && !P.fused && P.slices == 1 && P.hs && P.npass >= 2 &&
            P.cap <= (uint32_t)vxk::kGroupCapFast && (P.npass < 3 || P.D[2] <= (uint32_t)vxk::kPipeMaxBits) &&
            (1u << P.D[0]) >= zt)
            P.zt = zt;
    }
    // All three passes in the hash launches: slice i's second pass files
    // into regions of its own (one per first two digits, R[1] records each),
    // which launch i + 2 files by the third digit into the plot's shared
    // third-pass regions.  The third digit takes the filing kernel's 128
    // counters; tail_slices and batch_shared_hash keep the two-pass front.
    if (P.hq > 1 && P.npass == 3 && t->front_passes != 2 && P.zt == 1 && !P.fused && !t->batch_shared_hash &&
        P.D[2] <= (uint32_t)vxk::kPipeMaxBits) {
        const uint32_t b01 = P.D[0] + P.D[1];
        const double mean = (double)((((front_n + P.hq - 1) / P.hq) + (1ull << b01) - 1) >> b01);
        uint32_t r1 = (uint32_t)(mean + 8.0 * std::sqrt(mean)) + 64u;
        if (t->region_pct) r1 = std::max<uint32_t>(1, (uint32_t)((uint64_t)r1 * t->region_pct / 100));
        if (((uint64_t)r1 << b01) < (1ull << 31)) {
            P.deep = true;
            P.R[1] = r1;
        }
    }
    // Items of 4096 records (512-thread work-groups) when the launches file
    // three passes: each digit's runs are twice as long, which the
    // memory-bound launches need (k=31: 100.9 against 104.3 ms per plot);
    // with two passes both sizes measured alike.
    P.hsub = t->front_subtile ? t->front_subtile : (P.deep ? vxk::kHashPassWideSub : vxk::kHashScatterSub);
    if (staged >= 0 && P.hq > 1 && !P.deep) {
        // A staged plot that cannot file all three passes in its hash
        // launches hashes in one (with that plan's digits).
        vx_tuning one = *t;
        one.hash_slices = 1;
        return make_plan(p, &one, pl, records, max_k, staged);
    }
    if (staged >= 0 && !P.hs)
        return fail(VX_ERR_UNSUPPORTED,
                    "staged plots need two or more partition passes, a first digit of at most 8 bits and at "
                    "least chunk_bits, later digits of at most 9 bits, and chunks of fewer than 2^32 records");
    *pl = P;
    return VX_OK;
}

// Workspace regions (byte offsets from the workspace start, 256-aligned).
struct Layout {
    size_t header = 0;        // u32 words (kHdr*)
    size_t keys_no = 0;       // u64[n] nonce-order hashes (plot only)
    size_t scr_keys = 0;      // u64[n] partition scratch
    size_t scr_nonces = 0;    // u32[n]
    size_t hist[kMaxPasses] = {}, off[kMaxPasses] = {};  // u32[tiles][2^D]
    size_t gstart[kMaxPasses] = {};  // u32[2^(pre + D) + 1] group starts after each pass
    size_t ovf_list = 0;          // u32[2^G]
    size_t lbwords = 0;           // u64[2^G] look-back words of the fused sort + match
    size_t mcount = 0, mbase = 0; // u64[match chunks]: pair counts, Table-2 bases
    size_t pcnt = 0;              // u8[n]: pair count of each Table-1 record (255 = look again)
    size_t nonces_in = 0;         // u32[n]: nonces of a chunk's records (chunked plots)
    size_t reg_nonces = 0;        // u32[regions]: nonces of the even passes' regions (hs)
    // hs, per pass: u32[2^(pre + D)] region fill counts and bounds
    size_t fill[kMaxPasses] = {}, seg_lo[kMaxPasses] = {}, seg_hi[kMaxPasses] = {};
    size_t mpart = 0;             // u64[scan parts]
    size_t pipelist = 0;          // the work list of a k_pipe launch (plot)
    size_t total = 0;
};

// Workspace header: u32 words zeroed at the start of every call.
constexpr uint32_t kHeaderWords = 160;
constexpr uint32_t kHdrStatus = 0;       // device status bits
constexpr uint32_t kHdrFusedTicket = 2;  // group ticket of the fused sort + match
constexpr uint32_t kHdrAcc = 4;          // u64 (words 4, 5): Table-2 records of the slices scanned so far
constexpr uint32_t kHdrChunkCount = 6;   // u64 (words 6, 7): records a chunk's hash kept
constexpr uint32_t kHdrOvf = 8;          // per slice: oversized groups found
constexpr uint32_t kHdrSortTicket = 8 + kMaxSlices;       // per slice: group ticket of the sort
constexpr uint32_t kHdrEmitTicket = 8 + 2 * kMaxSlices;   // per slice: chunk ticket of the match
constexpr uint32_t kHdrHashPassTicket = 8 + 3 * kMaxSlices;  // per launch of a sliced hash
constexpr uint32_t kHdrPipeTicket = kHdrHashPassTicket + kMaxHashSlices + 2;  // per launch of a pipelined tail
constexpr uint32_t kHdrBatchTicket = kHdrPipeTicket + kMaxTailSlices + 2;  // fused launches of a batch
constexpr uint32_t kBatchTicketWords = kHeaderWords - kHdrBatchTicket;
static_assert(kBatchTicketWords >= 21, "a batch round needs up to 21 launches per plot");
constexpr uint32_t kLookbackSpinLimit = 1u << 20;

constexpr int kCallChunk = 4;        // internal: the workspace of vx_plot_chunk
constexpr int kCallStagedChunk = 5;  // internal: the workspace of vx_plot_staged_chunk
constexpr uint32_t kMaxChunkBits = 8;

uint32_t match_chunks(const Plan &P) { return (uint32_t)((P.n + (1ull << P.cb) - 1) >> P.cb); }

// A plan whose hash launches file all three passes (P.deep) keeps slice i's
// first-pass regions (pass 0) and second-pass regions (pass 1) in slot
// i % 2 of a two-slot ring each, in the scratch arrays: launch i writes the
// first-pass regions of slice i and the second-pass regions of slice i - 1,
// and reads those of slices i - 1 and i - 2, written by the launch before.
uint64_t ring_slot(const Plan &P, uint32_t pass) {
    return pass == 0 ? (uint64_t)P.R[0] << P.D[0] : (uint64_t)P.R[1] << (P.D[0] + P.D[1]);
}

uint32_t pass_tiles(const Plan &P, uint32_t i) {
    return i == 0 ? P.W : (1u << P.pre[i]) * P.Q[i];
}

Layout layout(const Plan &P, int which) {
    Layout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t o = at;
        at = align_up(at + bytes, 256);
        return o;
    };
    L.header = take(kHeaderWords * 4);
    const bool chunk = which == kCallChunk;
    const bool staged = which == kCallStagedChunk;
    if (chunk || staged) which = VX_CALL_PLOT;
    const bool sort = which == VX_CALL_BUCKET_SORT || which == VX_CALL_PLOT;
    const bool match = which == VX_CALL_MATCH || which == VX_CALL_PLOT;
    // A region-pass plot (P.hs) files the even passes (the first in the
    // hash kernel) into keys_no + reg_nonces and the odd ones into the
    // scratch arrays, each as fixed-size regions with slack; Table 1 is
    // written only by the group sort.  A staged chunk's first pass is in the
    // stage, and its later passes hold only the chunk's share of regions.
    const bool hs = which == VX_CALL_PLOT && !chunk && P.hs;
    const uint32_t cbits = staged ? (uint32_t)P.staged : 0;
    uint64_t cap_even = staged ? 0 : P.n, cap_odd = staged ? 0 : P.n;
    for (uint32_t i = staged ? 1 : 0; hs && !P.deep && i < P.npass; ++i) {
        const uint64_t c = ((uint64_t)P.R[i] << (P.pre[i] + P.D[i] - cbits)) * (i == 0 ? P.hq : 1);
        uint64_t &m = (i % 2 == 0) ? cap_even : cap_odd;
        m = std::max(m, c);
    }
    if (hs && P.deep) {
        // The third pass's regions; the first two passes' regions of two
        // slices at a time (ring_slot).  A staged chunk reads all of them
        // from the stage.
        cap_even = staged ? 0 : std::max<uint64_t>(P.n, (uint64_t)P.R[2] << P.G);
        cap_odd = staged ? 0 : 2 * (ring_slot(P, 0) + ring_slot(P, 1));
    }
    if (which == VX_CALL_PLOT) L.keys_no = take(cap_even * 8);
    if (hs) L.reg_nonces = take(cap_even * 4);
    for (uint32_t i = 0; hs && i < P.npass; ++i) {
        const size_t nr = (size_t)1 << (P.pre[i] + P.D[i]);
        L.fill[i] = take(i == 0 && P.hq > 1 ? (size_t)slice_fill_stride(P.D[0]) * P.hq * 4
                         : (i == 1 && P.deep ? nr * P.hq * 4 : nr * 4));
        L.seg_lo[i] = take(nr * 4);
        L.seg_hi[i] = take(nr * 4);
    }
    if (chunk) L.nonces_in = take(P.n * 4);
    const uint64_t scr = cap_odd;
    if (sort) {
        L.scr_keys = take(scr * 8);
        L.scr_nonces = take(scr * 4);
        for (uint32_t i = 0; i < P.npass; ++i) {
            const size_t cells = (size_t)pass_tiles(P, i) << P.D[i];
            L.hist[i] = take(cells * 4);
            L.off[i] = take(cells * 4);
            L.gstart[i] = take((((size_t)1 << (P.pre[i] + P.D[i])) + 1) * 4);
        }
        L.ovf_list = take((size_t)(1u << P.G) * 4);
        if (which == VX_CALL_PLOT) L.lbwords = take((size_t)(1u << P.G) * 8);
    }
    if (match) {
        const uint32_t nch = match_chunks(P);
        L.mcount = take((size_t)nch * 8);
        L.mbase = take((size_t)nch * 8);
        L.mpart = take((size_t)vxk::scan_parts(nch) * 8);
        if (which == VX_CALL_PLOT && !chunk && !staged) L.pipelist = take(sizeof(vxk::PipeList));
        L.pcnt = take(align_up(P.n, 4));
    }
    L.total = at;
    return L;
}

// A stage (vx_stage_plot): header words, the first pass's region fills and
// its regions (SoA).  A stage hashed in slices (P.deep) holds instead the
// third pass's region fills and regions (chunk c's regions from record
// c * 2^(G - chunk_bits) * R2 on), the second pass's per-slice region fills
// (the chunks' group starts come from them), the first pass's per-slice
// fills, and the two rings the hash launches file the first two passes
// through.
constexpr uint32_t kStageMagic = 0x56585354u;  // "VXST"
constexpr uint32_t kStageIdWords = 16;  // header words [1, 16): what the stage was made for
struct StageLayout {
    // u32[64]: [0] status; [1] magic, [2] k, [3] D0, [4] R0, [5] chunk_bits,
    // [6, 14) key words, [14] slices | deep << 8 | D1 << 16 | D2 << 24, [15] R2
    size_t header = 0;
    size_t fill = 0;    // u32[2^D0] (deep: u32[2^G], the third pass's)
    size_t keys = 0;    // u64[2^D0 * R0] (deep: u64[2^G * R2])
    size_t nonces = 0;  // u32[2^D0 * R0] (deep: u32[2^G * R2])
    size_t fill0 = 0, fill1 = 0;            // deep: per-slice first- and second-pass fills
    size_t ring_keys = 0, ring_nonces = 0;  // deep: two slots of each ring
    size_t total = 0;
};

void stage_id(const Plan &P, uint32_t chunk_bits, uint32_t id[kStageIdWords]) {
    memset(id, 0, kStageIdWords * 4);
    id[1] = kStageMagic;
    id[2] = P.k;
    id[3] = P.D[0];
    id[4] = P.R[0];
    id[5] = chunk_bits;
    for (int i = 0; i < 8; ++i) id[6 + i] = P.key_words[i];
    id[14] = P.hq | (P.deep ? 1u << 8 : 0u) | (P.D[1] << 16) | (P.D[2] << 24);
    id[15] = P.R[2];
}

StageLayout stage_layout(const Plan &P) {
    StageLayout S;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t o = at;
        at = align_up(at + bytes, 256);
        return o;
    };
    S.header = take(kHeaderWords * 4);
    if (P.deep) {
        const uint64_t recs = (uint64_t)P.R[2] << P.G;
        const uint64_t ring = 2 * (ring_slot(P, 0) + ring_slot(P, 1));
        S.fill = take((size_t)4 << P.G);
        S.fill0 = take((size_t)slice_fill_stride(P.D[0]) * P.hq * 4);
        S.fill1 = take(((size_t)P.hq << (P.D[0] + P.D[1])) * 4);
        S.keys = take(recs * 8);
        S.nonces = take(recs * 4);
        S.ring_keys = take(ring * 8);
        S.ring_nonces = take(ring * 4);
    } else {
        const uint64_t recs = (uint64_t)P.R[0] << P.D[0];
        S.fill = take((size_t)4 << P.D[0]);
        S.keys = take(recs * 8);
        S.nonces = take(recs * 4);
    }
    S.total = at;
    return S;
}

template <typename T>
T *at(void *ws, size_t off);
void set_frac(vxk::HashPassList &W);

// The stage of a plot hashed in slices with all three passes in the hash
// launches (P.deep): as run_sliced_front, in the stage's buffers, with one
// third-pass descriptor per chunk, so that chunk c's third-pass regions are
// its own (record indices below 2^32) and it can sort them alone.
vx_status stage_sliced_front(const Plan &P, const StageLayout &S, uint32_t cb, void *d_stage, hipStream_t s) {
    uint32_t *hdr = at<uint32_t>(d_stage, S.header);
    const uint32_t b01 = P.D[0] + P.D[1], sub = P.hsub;
    const uint32_t stride0 = slice_fill_stride(P.D[0]);
    uint32_t *fill0 = at<uint32_t>(d_stage, S.fill0), *fill1 = at<uint32_t>(d_stage, S.fill1);
    uint32_t *fill2 = at<uint32_t>(d_stage, S.fill);
    uint64_t *rk = at<uint64_t>(d_stage, S.ring_keys);
    uint32_t *rn = at<uint32_t>(d_stage, S.ring_nonces);
    const uint64_t slot0 = ring_slot(P, 0), slot1 = ring_slot(P, 1);
    VX_HIP(vxk::launch_fill_u32(fill0, (uint64_t)stride0 * P.hq, 0u, s), "reset");
    VX_HIP(vxk::launch_fill_u32(fill1, (uint64_t)P.hq << b01, 0u, s), "reset");
    VX_HIP(vxk::launch_fill_u32(fill2, 1ull << P.G, 0u, s), "reset");
    const uint32_t nch = 1u << cb, nin_c = 1u << (b01 - cb);
    const uint64_t creg = (uint64_t)P.R[2] << (P.G - cb);  // records of a chunk's third-pass regions
    for (uint32_t i = 0; i < P.hq + 2; ++i) {
        vxk::HashPassList W;
        memset(&W, 0, sizeof(W));
        W.sub = sub;
        if (i < P.hq) {
            vxk::HashSliceDesc &H = W.h[W.nh++];
            memcpy(H.key, P.key_words, sizeof(H.key));
            H.nonce0 = P.n * i / P.hq;
            H.n = P.n * (i + 1) / P.hq - H.nonce0;
            H.keys = rk + (i % 2) * slot0;
            H.nonces = rn + (i % 2) * slot0;
            H.fill = fill0 + (size_t)i * stride0;
            H.status = hdr + kHdrStatus;
            H.bits = P.D[0];
            H.R = P.R[0];
            H.items = (uint32_t)((H.n + sub - 1) / sub);
            W.h_items += H.items;
        }
        if (i >= 1 && i - 1 < P.hq) {  // slice i - 1 by the second digit
            const uint32_t j = i - 1, per = (P.R[0] + sub - 1) / sub;
            vxk::PassSliceDesc &Q = W.p[W.np++];
            Q.keys = rk + (j % 2) * slot0;
            Q.nonces = rn + (j % 2) * slot0;
            Q.fill = fill0 + (size_t)j * stride0;
            Q.out_keys = rk + 2 * slot0 + (j % 2) * slot1;
            Q.out_nonces = rn + 2 * slot0 + (j % 2) * slot1;
            Q.out_fill = fill1 + ((size_t)j << b01);
            Q.status = hdr + kHdrStatus;
            Q.R_in = P.R[0];
            Q.per = per;
            Q.shift = 64 - b01;
            Q.bits = P.D[1];
            Q.R_out = P.R[1];
            Q.items = (1u << P.D[0]) * per;
            W.p_items += Q.items;
        }
        if (i >= 2) {  // slice i - 2 by the third digit, chunk by chunk
            const uint32_t j = i - 2, per = (P.R[1] + sub - 1) / sub;
            for (uint32_t c = 0; c < nch; ++c) {
                vxk::PassSliceDesc &Q = W.p[W.np++];
                const uint64_t in0 = 2 * slot0 + (j % 2) * slot1 + (uint64_t)c * nin_c * P.R[1];
                Q.keys = rk + in0;
                Q.nonces = rn + in0;
                Q.fill = fill1 + ((size_t)j << b01) + (size_t)c * nin_c;
                Q.out_keys = at<uint64_t>(d_stage, S.keys) + c * creg;
                Q.out_nonces = at<uint32_t>(d_stage, S.nonces) + c * creg;
                Q.out_fill = fill2 + ((size_t)c << (P.G - cb));
                Q.status = hdr + kHdrStatus;
                Q.R_in = P.R[1];
                Q.per = per;
                Q.shift = 64 - P.G;
                Q.bits = P.D[2];
                Q.R_out = P.R[2];
                Q.items = nin_c * per;
                W.p_items += Q.items;
            }
        }
        set_frac(W);
        VX_HIP(vxk::launch_hash_pass(W, hdr + kHdrHashPassTicket + i, s), "stage hash");
    }
    return VX_OK;
}

// Records ev[i] on s when an event array is given (stage timing).
inline hipError_t mark(hipEvent_t *ev, int i, hipStream_t s) {
    return ev ? hipEventRecord(ev[i], s) : hipSuccess;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Where partition pass i reads and writes.  Contiguous passes alternate
// between Table 1 and the scratch arrays so that the last one lands in
// Table 1, where groups are then sorted in place; region passes (P.hs)
// alternate between keys_no + reg_nonces and the scratch arrays, and the
// group sort gathers into Table 1.
struct PassBufs {
    const uint64_t *in_k;
    const uint32_t *in_n;  // NULL: nonce = index (the nonce-order keys)
    uint64_t *out_k;
    uint32_t *out_n;
};

PassBufs pass_bufs(const Plan &P, const Layout &L, void *ws, const uint64_t *keys_no, uint64_t *t1_keys,
                   uint32_t *t1_nonces, uint32_t i, const uint32_t *nonces_in = nullptr) {
    uint64_t *scr_k = at<uint64_t>(ws, L.scr_keys);
    uint32_t *scr_n = at<uint32_t>(ws, L.scr_nonces);
    auto to_t1 = [&](uint32_t j) { return ((P.npass - 1 - j) % 2) == 0; };
    PassBufs B;
    if (P.hs) {
        // Even passes (the first in the hash kernel) fill regions in keys_no +
        // reg_nonces, odd ones in the scratch arrays; each reads the other.
        uint64_t *reg_k = at<uint64_t>(ws, L.keys_no);
        uint32_t *reg_n = at<uint32_t>(ws, L.reg_nonces);
        B.in_k = i == 0 ? nullptr : (i % 2 ? reg_k : scr_k);
        B.in_n = i == 0 ? nullptr : (i % 2 ? reg_n : scr_n);
        B.out_k = i % 2 ? scr_k : reg_k;
        B.out_n = i % 2 ? scr_n : reg_n;
        return B;
    }
    if (i == 0) {
        B.in_k = keys_no;
        B.in_n = nonces_in;
    } else {
        B.in_k = to_t1(i - 1) ? t1_keys : scr_k;
        B.in_n = to_t1(i - 1) ? t1_nonces : scr_n;
    }
    B.out_k = to_t1(i) ? t1_keys : scr_k;
    B.out_n = to_t1(i) ? t1_nonces : scr_n;
    return B;
}

// After a region pass i >= 1 over input segments [sa, sb): the clamp of its
// regions' counts into their bounds, and their scan (one row per segment, on
// top of the segments' bases) into the group starts.
vx_status claimed_regions(const Plan &P, const Layout &L, void *ws, uint32_t i, uint32_t sa, uint32_t sb,
                          hipStream_t s, uint32_t origin = 0) {
    const uint32_t nd = 1u << P.D[i];
    const uint32_t nseg = sb - sa;
    const uint32_t *base = at<uint32_t>(ws, L.gstart[i - 1]) + sa;
    uint32_t *off = at<uint32_t>(ws, L.off[i]) + (size_t)sa * P.Q[i] * nd;
    uint32_t *gst = at<uint32_t>(ws, L.gstart[i]) + (size_t)sa * nd;
    uint32_t *fill = at<uint32_t>(ws, L.fill[i]) + (size_t)sa * nd;
    VX_HIP(vxk::launch_region_bounds(fill, (sa - origin) * nd, nseg * nd, P.R[i],
                                     at<uint32_t>(ws, L.seg_lo[i]) + sa * nd,
                                     at<uint32_t>(ws, L.seg_hi[i]) + sa * nd, s),
           "pass regions");
    VX_HIP(vxk::launch_colscan(fill, off, nseg, 1, nd, base, gst, nseg * nd, (uint32_t)P.n, s), "pass scan");
    return VX_OK;
}

// Pass i >= 1 over its input segments [sa, sb) (the groups of pass i - 1).
// A region-pass plan (P.hs) reads the previous pass's regions and claims
// room in its own: the scatter, the clamp of the region counts, and their
// scan (one row per segment, on top of the segments' bases) into the group
// starts.  Otherwise segments lie back to back at the previous pass's group
// starts: per-tile histograms, their scan inside each segment, the scatter.
//
// origin: the segment whose regions start the output buffer (a staged chunk
// holds only its own share of regions; 0 otherwise).
vx_status run_pass(const Plan &P, const Layout &L, void *ws, const PassBufs &B, uint32_t i, uint32_t sa,
                   uint32_t sb, hipStream_t s, uint32_t origin = 0) {
    const uint32_t nd = 1u << P.D[i];
    const uint32_t shift = 64 - P.pre[i] - P.D[i];
    const uint32_t q = P.Q[i];
    const uint32_t nseg = sb - sa;
    const uint32_t *base = at<uint32_t>(ws, L.gstart[i - 1]) + sa;
    uint32_t *off = at<uint32_t>(ws, L.off[i]) + (size_t)sa * q * nd;
    uint32_t *gst = at<uint32_t>(ws, L.gstart[i]) + (size_t)sa * nd;
    if (P.hs) {
        const uint32_t *seg = at<uint32_t>(ws, L.seg_lo[i - 1]) + sa;
        const uint32_t *seg_end = at<uint32_t>(ws, L.seg_hi[i - 1]) + sa;
        uint32_t *fill = at<uint32_t>(ws, L.fill[i]) + (size_t)sa * nd;
        const uint64_t first = (uint64_t)(sa - origin) * nd * P.R[i];
        VX_HIP(vxk::launch_scatter_claim(B.in_k, B.in_n, B.out_k + first, B.out_n + first, seg, seg_end, nseg, q,
                                         shift, P.D[i], fill, P.R[i], at<uint32_t>(ws, L.header) + kHdrStatus, s),
               "pass scatter");
        return claimed_regions(P, L, ws, i, sa, sb, s, origin);
    }
    uint32_t *hist = at<uint32_t>(ws, L.hist[i]) + (size_t)sa * q * nd;
    VX_HIP(vxk::launch_hist_segments(B.in_k, base, nullptr, nseg, q, shift, P.D[i], hist, s), "pass histogram");
    VX_HIP(vxk::launch_colscan(hist, off, nseg, q, nd, base, gst, nseg * nd, (uint32_t)P.n, s), "pass scan");
    VX_HIP(vxk::launch_scatter_segments(B.in_k, B.in_n, B.out_k, B.out_n, off, base, nullptr, nseg, q, shift,
                                        P.D[i], s),
           "pass scatter");
    return VX_OK;
}

// Partition passes [0, npass_run).  Pass 0 reads the nonce-order keys (its
// histogram comes from the hash kernel in a plot, or from a histogram pass
// over caller keys).
// The passes a plot's hash launches file: none (a separate hash), the first
// (the hash kernel's own), or the first two (sliced or fused launches).
uint32_t hash_passes(const Plan &P) { return P.hs ? (P.hq > 1 ? (P.deep ? 3 : 2) : 1) : 0; }

vx_status run_partition(const Plan &P, const Layout &L, void *ws, const uint64_t *keys_no,
                        bool hist_done, uint64_t *t1_keys, uint32_t *t1_nonces, uint32_t npass_run,
                        hipStream_t s, hipEvent_t *ev, const uint32_t *nonces_in = nullptr,
                        uint32_t first = UINT32_MAX) {
    if (first == UINT32_MAX) first = hash_passes(P);
    if (first >= npass_run) VX_HIP(mark(ev, 3, s), "event");
    for (uint32_t i = first; i < npass_run; ++i) {
        const PassBufs B = pass_bufs(P, L, ws, keys_no, t1_keys, t1_nonces, i, nonces_in);
        if (i == 0) {
            uint32_t *hist = at<uint32_t>(ws, L.hist[0]), *off = at<uint32_t>(ws, L.off[0]);
            uint32_t *gst = at<uint32_t>(ws, L.gstart[0]);
            const uint32_t nd = 1u << P.D[0];
            const uint32_t shift = 64 - P.D[0];
            if (!hist_done)
                VX_HIP(vxk::launch_hist_chunks(B.in_k, P.n, P.W, P.chunk1, shift, P.D[0], hist, s),
                       "pass-0 histogram");
            VX_HIP(vxk::launch_colscan(hist, off, 1, P.W, nd, nullptr, gst, nd, (uint32_t)P.n, s), "pass-0 scan");
            VX_HIP(vxk::launch_scatter_chunks(B.in_k, B.in_n, B.out_k, B.out_n, off, P.n, P.W, P.chunk1, shift,
                                              P.D[0], s),
                   "pass-0 scatter");
        } else {
            vx_status st = run_pass(P, L, ws, B, i, 0, 1u << P.pre[i], s);
            if (st != VX_OK) return st;
        }
        VX_HIP(mark(ev, i == 0 ? 2 : 3, s), "event");
    }
    if (npass_run == 1 && first < npass_run) VX_HIP(mark(ev, 3, s), "event");
    return VX_OK;
}

// The hash and the first two partition passes of a plot hashed in P.hq
// nonce slices.  Launch i hashes slice i and files it by the first digit
// into its own regions, while its other work-groups file the regions of
// slice i - 1 (written by launch i - 1) by the second digit into the plot's
// second-pass regions, shared by all slices.  Then the first digit's group
// starts over all slices, and the second pass's region bounds and group
// starts.
// Slice i of a plan whose hash files two passes (P.hs, two or more passes,
// both digits within the sliced kernel's width; P.hq slices, one when the
// plan is not sliced): its hash (first digit, into the slice's own regions)
// and its second pass (over those regions, into the plot's second-pass
// regions).
bool front_fusable(const Plan &P) {
    return P.hs && !P.deep && P.npass >= 2 && P.D[0] <= (uint32_t)vxk::kHashPassMaxBits &&
           P.D[1] <= (uint32_t)vxk::kHashPassMaxBits;
}

uint32_t front_fill_stride(const Plan &P) { return P.hq > 1 ? slice_fill_stride(P.D[0]) : 1u << P.D[0]; }

// Where slice i's first-pass regions live: slot i of the even-pass region
// arrays, or (P.deep) ring slot i % 2 in the scratch arrays.
uint64_t *first_keys(const Plan &P, const Layout &L, void *ws, uint32_t i) {
    return P.deep ? at<uint64_t>(ws, L.scr_keys) + (i % 2) * ring_slot(P, 0)
                  : at<uint64_t>(ws, L.keys_no) + i * ring_slot(P, 0);
}

uint32_t *first_nonces(const Plan &P, const Layout &L, void *ws, uint32_t i) {
    return P.deep ? at<uint32_t>(ws, L.scr_nonces) + (i % 2) * ring_slot(P, 0)
                  : at<uint32_t>(ws, L.reg_nonces) + i * ring_slot(P, 0);
}

vxk::HashSliceDesc hash_slice(const Plan &P, const Layout &L, void *ws, uint32_t i,
                              uint32_t sub = vxk::kHashScatterSub) {
    vxk::HashSliceDesc H;
    memset(&H, 0, sizeof(H));
    memcpy(H.key, P.key_words, sizeof(H.key));
    H.nonce0 = P.n * i / P.hq;
    H.n = P.n * (i + 1) / P.hq - H.nonce0;
    H.keys = first_keys(P, L, ws, i);
    H.nonces = first_nonces(P, L, ws, i);
    H.fill = at<uint32_t>(ws, L.fill[0]) + (size_t)i * front_fill_stride(P);
    H.status = at<uint32_t>(ws, L.header) + kHdrStatus;
    H.bits = P.D[0];
    H.R = P.R[0];
    H.items = (uint32_t)((H.n + sub - 1) / sub);
    return H;
}

vxk::PassSliceDesc pass_slice(const Plan &P, const Layout &L, void *ws, uint32_t i,
                              uint32_t sub = vxk::kHashScatterSub) {
    vxk::PassSliceDesc Q;
    memset(&Q, 0, sizeof(Q));
    const uint32_t per = (P.R[0] + sub - 1) / sub;
    Q.keys = first_keys(P, L, ws, i);
    Q.nonces = first_nonces(P, L, ws, i);
    Q.fill = at<uint32_t>(ws, L.fill[0]) + (size_t)i * front_fill_stride(P);
    if (P.deep) {
        // The slice's own second-pass regions (ring slot i % 2, counters of
        // its own).
        const uint64_t o = 2 * ring_slot(P, 0) + (i % 2) * ring_slot(P, 1);
        Q.out_keys = at<uint64_t>(ws, L.scr_keys) + o;
        Q.out_nonces = at<uint32_t>(ws, L.scr_nonces) + o;
        Q.out_fill = at<uint32_t>(ws, L.fill[1]) + ((size_t)i << (P.D[0] + P.D[1]));
    } else {
        Q.out_keys = at<uint64_t>(ws, L.scr_keys);
        Q.out_nonces = at<uint32_t>(ws, L.scr_nonces);
        Q.out_fill = at<uint32_t>(ws, L.fill[1]);
    }
    Q.status = at<uint32_t>(ws, L.header) + kHdrStatus;
    Q.R_in = P.R[0];
    Q.per = per;
    Q.shift = 64 - P.D[0] - P.D[1];
    Q.bits = P.D[1];
    Q.R_out = P.R[1];
    Q.items = (1u << P.D[0]) * per;
    return Q;
}

// The third pass of slice i (P.deep): its second-pass regions (ring slot
// i % 2), filed by the third digit into the plot's third-pass regions,
// shared by all slices, from which the group sort gathers.
vxk::PassSliceDesc third_slice(const Plan &P, const Layout &L, void *ws, uint32_t i, uint32_t sub) {
    vxk::PassSliceDesc Q;
    memset(&Q, 0, sizeof(Q));
    const uint32_t b01 = P.D[0] + P.D[1];
    const uint32_t per = (P.R[1] + sub - 1) / sub;
    const uint64_t o = 2 * ring_slot(P, 0) + (i % 2) * ring_slot(P, 1);
    Q.keys = at<uint64_t>(ws, L.scr_keys) + o;
    Q.nonces = at<uint32_t>(ws, L.scr_nonces) + o;
    Q.fill = at<uint32_t>(ws, L.fill[1]) + ((size_t)i << b01);
    Q.out_keys = at<uint64_t>(ws, L.keys_no);
    Q.out_nonces = at<uint32_t>(ws, L.reg_nonces);
    Q.out_fill = at<uint32_t>(ws, L.fill[2]);
    Q.status = at<uint32_t>(ws, L.header) + kHdrStatus;
    Q.R_in = P.R[1];
    Q.per = per;
    Q.shift = 64 - b01 - P.D[2];
    Q.bits = P.D[2];
    Q.R_out = P.R[2];
    Q.items = (1u << b01) * per;
    return Q;
}

// Proportions of a launch's two kinds of items (k_hash_pass).
void set_frac(vxk::HashPassList &W) {
    const uint64_t nt = (uint64_t)W.h_items + W.p_items;
    const uint64_t num = (uint64_t)W.h_items << 32;
    W.h_frac = nt ? num / nt + (num % nt ? 1 : 0) : 0;
}

// After every slice's second pass: the first digit's group starts over all
// slices, then the second pass's region bounds and group starts.
vx_status finish_front(const Plan &P, const Layout &L, void *ws, hipStream_t s) {
    const uint32_t nd0 = 1u << P.D[0];
    VX_HIP(vxk::launch_region_scan_slices(at<uint32_t>(ws, L.fill[0]), P.hq, front_fill_stride(P), nd0, P.R[0],
                                          at<uint32_t>(ws, L.gstart[0]), s),
           "region scan");
    return claimed_regions(P, L, ws, 1, 0, nd0, s);
}

// P.deep: after every slice's third pass, the second pass's group starts
// (summed over the slices' own regions), then the third pass's region
// bounds and group starts on top of them.
vx_status finish_deep_front(const Plan &P, const Layout &L, void *ws, hipStream_t s) {
    const uint32_t nd01 = 1u << (P.D[0] + P.D[1]);
    VX_HIP(vxk::launch_region_scan_slices(at<uint32_t>(ws, L.fill[1]), P.hq, nd01, nd01, P.R[1],
                                          at<uint32_t>(ws, L.gstart[1]), s),
           "region scan");
    return claimed_regions(P, L, ws, 2, 0, nd01, s);
}

// Launch i hashes slice i and files the regions of slice i - 1 by the
// second digit (and, P.deep, those of slice i - 2 by the third), each kind
// reading what the launch before wrote.
vx_status run_sliced_front(const Plan &P, const Layout &L, void *ws, hipStream_t s, hipEvent_t *ev) {
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    const uint32_t lag = P.deep ? 2 : 1;
    for (uint32_t i = 0; i < P.hq + lag; ++i) {
        vxk::HashPassList W;
        memset(&W, 0, sizeof(W));
        W.sub = P.hsub;
        if (i < P.hq) {
            W.h[W.nh++] = hash_slice(P, L, ws, i, P.hsub);
            W.h_items += W.h[0].items;
        }
        if (i >= 1 && i - 1 < P.hq) {
            W.p[W.np] = pass_slice(P, L, ws, i - 1, P.hsub);
            W.p_items += W.p[W.np++].items;
        }
        if (P.deep && i >= 2) {
            W.p[W.np] = third_slice(P, L, ws, i - 2, P.hsub);
            W.p_items += W.p[W.np++].items;
        }
        set_frac(W);
        VX_HIP(vxk::launch_hash_pass(W, hdr + kHdrHashPassTicket + i, s), "sliced hash");
    }
    VX_HIP(mark(ev, 1, s), "event");
    vx_status st = P.deep ? finish_deep_front(P, L, ws, s) : finish_front(P, L, ws, s);
    if (st != VX_OK) return st;
    VX_HIP(mark(ev, 2, s), "event");
    return VX_OK;
}

// Sort of the partitioned groups [g0, g0 + gcount) (+ oversized groups)
// into Table 1, with their bucket offsets; `slot` picks the slice's header
// words.  Groups are sorted in place, or (region-pass plans) gathered from
// the last pass's regions.  pcnt (may be NULL): the sort also stores every
// record's pair count (one byte) while the group is in LDS.  sums: it also
// adds the counts up per match chunk (L.mcount, zeroed here first), so that
// the match needs no pass over the count bytes; only when the sorted groups
// hold every record of the table.  (The reductions cost the sort more than
// the separate pass over the count bytes takes, measured at k=31: 15.6 ms
// against 12.9 + 0.8 ms; the pipelined tail uses them, the rest does not.)
vx_status run_group_sort(const Plan &P, const Layout &L, void *ws, uint64_t *t1_keys, uint32_t *t1_nonces,
                         uint32_t *offsets, uint8_t *pcnt, uint32_t g0, uint32_t gcount, uint32_t slot,
                         hipStream_t s, bool sums = false, const uint64_t *regions_k = nullptr,
                         const uint32_t *regions_n = nullptr) {
    uint64_t *csum = nullptr;
    if (sums && pcnt) {
        csum = at<uint64_t>(ws, L.mcount);
        VX_HIP(vxk::launch_zero_u64(csum, match_chunks(P), s), "zero chunk sums");
    }
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    const uint32_t last = P.npass - 1;
    const uint32_t *gstart = at<uint32_t>(ws, L.gstart[last]);
    uint32_t *ovf_list = at<uint32_t>(ws, L.ovf_list) + g0;
    const uint64_t *in_k = nullptr;
    const uint32_t *in_n = nullptr, *in_lo = nullptr, *in_hi = nullptr;
    if (P.hs) {
        const PassBufs B = pass_bufs(P, L, ws, nullptr, t1_keys, t1_nonces, last);
        in_k = regions_k ? regions_k : B.out_k;  // (a staged chunk's regions are in the stage)
        in_n = regions_k ? regions_n : B.out_n;
        in_lo = at<uint32_t>(ws, L.seg_lo[last]);
        in_hi = at<uint32_t>(ws, L.seg_hi[last]);
    }
    VX_HIP(vxk::launch_groupsort(t1_keys, t1_nonces, in_k, in_n, in_lo, in_hi, gstart, P.G, P.cap, offsets, (uint32_t)P.n,
                                 hdr + kHdrOvf + slot, ovf_list, P.T, pcnt, g0, gcount,
                                 hdr + kHdrSortTicket + slot, csum, P.cb, s),
           "group sort");
    VX_HIP(vxk::launch_group_fallback(t1_keys, t1_nonces, in_k, in_n, in_lo, in_hi, at<uint64_t>(ws, L.scr_keys),
                                      at<uint32_t>(ws, L.scr_nonces), gstart, P.G, offsets, hdr + kHdrOvf + slot,
                                      ovf_list, hdr + kHdrStatus, P.T, pcnt, csum, P.cb, s),
           "group sort fallback");
    return VX_OK;
}

// Match and Table-2 hashing of the chunks owned by records [*r_lo, *r_hi)
// (NULL: all), whose count bytes are in the workspace: chunk sums (unless
// sums_ready: the sort or the match count made them), Table-2 bases (a
// device scan over all chunks when unsliced, else a ranged scan that carries
// the running total), then the match kernel.
vx_status run_match(const Plan &P, const Layout &L, void *ws, const uint64_t *t1_keys,
                    const uint32_t *t1_nonces, vx_t2_record *t2, uint64_t cap, uint64_t *t2_count,
                    const uint32_t *r_lo, const uint32_t *r_hi, uint32_t last, uint32_t slot, uint32_t wg_per_cu,
                    hipStream_t s, hipEvent_t *ev = nullptr, bool sums_ready = false) {
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    uint64_t *cnt = at<uint64_t>(ws, L.mcount), *base = at<uint64_t>(ws, L.mbase);
    uint8_t *pcnt = at<uint8_t>(ws, L.pcnt);
    const uint32_t nch = match_chunks(P);
    if (!sums_ready)
        VX_HIP(vxk::launch_chunk_sums(pcnt, t1_keys, (uint32_t)P.n, P.cb, P.T, cnt, r_lo, r_hi, last, nch, s),
               "chunk pair sums");
    if (!r_lo) {
        VX_HIP(vxk::launch_scan_u64(cnt, nch, base, at<uint64_t>(ws, L.mpart), t2_count, s), "match scan");
    } else {
        VX_HIP(vxk::launch_scan_range(cnt, base, (uint32_t)P.n, P.cb, r_lo, r_hi, last,
                                      reinterpret_cast<uint64_t *>(hdr + kHdrAcc), t2_count, s),
               "match scan");
    }
    VX_HIP(mark(ev, 5, s), "event");
    VX_HIP(vxk::launch_match_emit(P.key_words, t1_keys, t1_nonces, pcnt, (uint32_t)P.n, P.cb, P.T, base, t2, cap,
                                  r_lo, r_hi, last, nch, wg_per_cu, hdr + kHdrEmitTicket + slot, s),
           "match emit");
    VX_HIP(mark(ev, 6, s), "event");
    return VX_OK;
}

// The plot's work after its first two partition passes, software-pipelined
// over P.zt slices of the second pass's regions (of the groups, when there
// are only two passes).  Launch i of k_pipe files slice i by the third
// digit, sorts slice i - 1 and matches slice i - 2 (fewer stages without a
// third pass); between launches come the third pass's region bounds and
// group starts of slice i, the fallback sort of slice i - 1's oversized
// groups, and the Table-2 bases of the match chunks that slice i - 1 owns
// (a ranged scan carrying the running total; the last one stores |T2|).
// The sort adds each chunk's pair count (csum), so no pass over the count
// bytes is needed.  A slice's groups end at bucket boundaries, so a chunk's
// partners lie in its own slice or an earlier one, all sorted by then.
vx_status run_pipe_tail(const Plan &P, const Layout &L, void *ws, const vx_plot_buffers *b, hipStream_t s) {
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    const uint32_t last = P.npass - 1;
    const bool p3 = P.npass == 3;
    const uint32_t N1 = 1u << (P.pre[1] + P.D[1]);
    const uint32_t Z = P.zt;
    const uint32_t gper = p3 ? 1u << P.D[2] : 1u;
    const uint32_t *gst1 = at<uint32_t>(ws, L.gstart[1]);
    uint64_t *csum = at<uint64_t>(ws, L.mcount), *base = at<uint64_t>(ws, L.mbase);
    uint8_t *pcnt = at<uint8_t>(ws, L.pcnt);
    uint32_t *ovf_list = at<uint32_t>(ws, L.ovf_list);
    VX_HIP(vxk::launch_zero_u64(csum, match_chunks(P), s), "zero chunk sums");
    const PassBufs Bl = pass_bufs(P, L, ws, nullptr, b->t1_keys, b->t1_nonces, last);
    const PassBufs B2 = pass_bufs(P, L, ws, nullptr, b->t1_keys, b->t1_nonces, p3 ? 2 : last);
    const uint32_t per = (P.R[1] + vxk::kPipeSub - 1) / vxk::kPipeSub;
    vxk::PipeList *dl = at<vxk::PipeList>(ws, L.pipelist);
    const uint32_t off_s = p3 ? 1 : 0, off_m = off_s + 1;
    // Slices are whole first-pass segments (2^D[1] second-pass regions
    // each): a segment's Table-1 span is its first-pass count, which also
    // covers the holes a region overflow leaves after its groups, so the
    // segments' capacity bounds the match chunks a slice owns.
    const uint32_t N0 = 1u << P.D[0];
    auto seg_cut = [&](uint32_t j) { return (uint32_t)((uint64_t)N0 * j / Z); };
    auto cut = [&](uint32_t j) { return seg_cut(j) << P.D[1]; };
    (void)N1;
    const vxk::SortArgs sa{b->t1_keys, b->t1_nonces,
                           vxk::GroupIn{Bl.out_k, Bl.out_n, at<uint32_t>(ws, L.seg_lo[last]),
                                        at<uint32_t>(ws, L.seg_hi[last])},
                           at<uint32_t>(ws, L.gstart[last]), b->bucket_offsets, nullptr, nullptr, pcnt,
                           reinterpret_cast<unsigned long long *>(csum), P.T, P.G, P.cap, (uint32_t)P.n, P.cb};
    vxk::MatchArgs ma{{}, b->t1_keys, b->t1_nonces, pcnt, base, reinterpret_cast<uint4 *>(b->t2), b->t2_capacity,
                      P.T, (uint32_t)P.n, P.cb};
    memcpy(ma.key, P.key_words, sizeof(ma.key));
    for (uint32_t i = 0; i < Z + off_m; ++i) {
        vxk::PipeList W;
        memset(&W, 0, sizeof(W));
        if (p3 && i < Z) {  // the third pass over slice i
            const uint32_t a = cut(i), e = cut(i + 1);
            vxk::PassSliceDesc &Q = W.p[W.n[1]++];
            Q.keys = B2.in_k + (uint64_t)a * P.R[1];
            Q.nonces = B2.in_n + (uint64_t)a * P.R[1];
            Q.fill = at<uint32_t>(ws, L.fill[1]) + a;
            Q.out_keys = B2.out_k;
            Q.out_nonces = B2.out_n;
            Q.out_fill = at<uint32_t>(ws, L.fill[2]);
            Q.status = hdr + kHdrStatus;
            Q.R_in = P.R[1];
            Q.per = per;
            Q.shift = 64 - P.pre[2] - P.D[2];
            Q.bits = P.D[2];
            Q.R_out = P.R[2];
            Q.items = (e - a) * per;
            Q.r0 = a;
            W.items[1] += Q.items;
        }
        if (i >= off_s && i - off_s < Z) {  // the sort of slice j
            const uint32_t j = i - off_s, a = cut(j), e = cut(j + 1);
            vxk::PipeSortDesc &D = W.s[W.n[2]++];
            D.a = sa;
            D.a.ovf_count = hdr + kHdrOvf + j;
            D.a.ovf_list = ovf_list + a * gper;
            D.g0 = a * gper;
            D.items = (e - a) * gper;
            W.items[2] += D.items;
        }
        if (i >= off_m) {  // the match of slice j
            const uint32_t j = i - off_m, a = cut(j), e = cut(j + 1);
            vxk::PipeMatchDesc &M = W.m[W.n[3]++];
            M.a = ma;
            M.r_lo = gst1 + a;
            M.r_hi = gst1 + e;
            M.last = j + 1 == Z;
            // The slice's Table-1 span fits its segments' first-pass regions
            // (P.hq of R[0] records each); its chunks are at most one more
            // than that span fills.
            const uint64_t span = (uint64_t)(seg_cut(j + 1) - seg_cut(j)) * P.hq * P.R[0];
            const uint64_t maxrec = std::min<uint64_t>(P.n, span);
            M.items = (uint32_t)(maxrec >> P.cb) + 2;
            W.items[3] += M.items;
        }
        uint64_t rest = (uint64_t)W.items[0] + W.items[1] + W.items[2] + W.items[3];
        for (int r = 0; r < 3; ++r) {
            const uint64_t num = (uint64_t)W.items[r] << 32;
            W.frac[r] = rest ? num / rest + (num % rest ? 1 : 0) : 0;
            rest -= W.items[r];
        }
        VX_HIP(vxk::launch_pipe(W, dl, hdr + kHdrPipeTicket + i, s), "pipelined tail");
        if (p3 && i < Z) {
            vx_status st = claimed_regions(P, L, ws, 2, cut(i), cut(i + 1), s);
            if (st != VX_OK) return st;
        }
        if (i >= off_s && i - off_s < Z) {
            const uint32_t j = i - off_s, a = cut(j), e = cut(j + 1);
            VX_HIP(vxk::launch_group_fallback(b->t1_keys, b->t1_nonces, Bl.out_k, Bl.out_n,
                                              at<uint32_t>(ws, L.seg_lo[last]), at<uint32_t>(ws, L.seg_hi[last]),
                                              at<uint64_t>(ws, L.scr_keys), at<uint32_t>(ws, L.scr_nonces),
                                              at<uint32_t>(ws, L.gstart[last]), P.G, b->bucket_offsets,
                                              hdr + kHdrOvf + j, ovf_list + a * gper, hdr + kHdrStatus, P.T, pcnt,
                                              csum, P.cb, s),
                   "group sort fallback");
            VX_HIP(vxk::launch_scan_range(csum, base, (uint32_t)P.n, P.cb, gst1 + a, gst1 + e, j + 1 == Z,
                                          reinterpret_cast<uint64_t *>(hdr + kHdrAcc), b->t2_count, s),
                   "match scan");
        }
    }
    return VX_OK;
}

// Streams and events for pipelined plots, per device, created at default
// priority on first use.  A plot takes the next of a few stream slots, so
// plots enqueued on different caller streams rarely share one.
constexpr int kPipeSlots = 4;

struct Pipe {
    std::mutex mu;
    bool ready = false;
    uint32_t next = 0;
    hipStream_t y[kPipeSlots] = {};
    hipEvent_t ev[kPipeSlots][kMaxSlices + 1] = {};
};

constexpr int kMaxDevices = 64;
Pipe g_pipe[kMaxDevices];
std::mutex g_pipe_mu;

vx_status pipe_for_current_device(Pipe **out) {
    int dev = 0;
    VX_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(VX_ERR_UNSUPPORTED, "device index out of range");
    Pipe &Q = g_pipe[dev];
    std::lock_guard<std::mutex> guard(g_pipe_mu);
    if (!Q.ready) {
        for (int l = 0; l < kPipeSlots; ++l) {
            VX_HIP(hipStreamCreateWithFlags(&Q.y[l], hipStreamNonBlocking), "pipeline stream");
            for (uint32_t i = 0; i <= kMaxSlices; ++i)
                VX_HIP(hipEventCreateWithFlags(&Q.ev[l][i], hipEventDisableTiming), "pipeline event");
        }
        Q.ready = true;
    }
    *out = &Q;
    return VX_OK;
}

// The plot after its first partition pass, software-pipelined over slices
// of the first pass's segments.  Slice i's later passes and group sort run
// on the caller's stream; its chunk sums, Table-2 scan and match run on a
// second stream as soon as that sort is done, while the caller's stream
// already partitions and sorts slice i + 1.  The match is bound by the
// vector ALUs and the partition and sort by memory and LDS, so the two
// streams share each CU (the match takes at most two work-groups per CU;
// the persistent kernels take work from tickets, so work-groups that start
// late take less).  A slice owns the match chunks whose last record it
// holds; those chunks and their partners are final once its sort is done,
// because every earlier slice was sorted before it on the same stream.
vx_status run_pipelined(const Plan &P, const Layout &L, void *ws, const vx_plot_buffers *b,
                        const uint64_t *keys_no, hipStream_t s, hipEvent_t *ev) {
    Pipe *Q = nullptr;
    vx_status st = pipe_for_current_device(&Q);
    if (st != VX_OK) return st;
    std::lock_guard<std::mutex> guard(Q->mu);
    const int l = (int)(Q->next++ % kPipeSlots);
    hipStream_t y = Q->y[l];
    const uint32_t NS = 1u << P.D[0];
    const uint32_t S = P.slices;
    const uint32_t *gst0 = at<uint32_t>(ws, L.gstart[0]);
    uint8_t *pcnt = at<uint8_t>(ws, L.pcnt);
    VX_HIP(mark(ev, 3, s), "event");
    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t a = (uint32_t)((uint64_t)NS * i / S), e = (uint32_t)((uint64_t)NS * (i + 1) / S);
        for (uint32_t p = 1; p < P.npass; ++p) {
            const uint32_t sh = P.pre[p] - P.D[0];
            st = run_pass(P, L, ws, pass_bufs(P, L, ws, keys_no, b->t1_keys, b->t1_nonces, p), p, a << sh,
                          e << sh, s);
            if (st != VX_OK) return st;
        }
        const uint32_t gsh = P.G - P.D[0];
        st = run_group_sort(P, L, ws, b->t1_keys, b->t1_nonces, b->bucket_offsets, pcnt, a << gsh,
                            (e - a) << gsh, i, s);
        if (st != VX_OK) return st;
        VX_HIP(hipEventRecord(Q->ev[l][i], s), "slice event");
        VX_HIP(hipStreamWaitEvent(y, Q->ev[l][i], 0), "slice wait");
        st = run_match(P, L, ws, b->t1_keys, b->t1_nonces, b->t2, b->t2_capacity, b->t2_count, gst0 + a,
                       gst0 + e, i + 1 == S, i, 2, y);
        if (st != VX_OK) return st;
    }
    VX_HIP(mark(ev, 4, s), "event");
    VX_HIP(mark(ev, 5, s), "event");
    VX_HIP(hipEventRecord(Q->ev[l][kMaxSlices], y), "pipeline join");
    VX_HIP(hipStreamWaitEvent(s, Q->ev[l][kMaxSlices], 0), "pipeline join wait");
    VX_HIP(mark(ev, 6, s), "event");
    return VX_OK;
}

vx_status check_ws(const Layout &L, const void *ws, size_t bytes) {
    if (!ws) return fail(VX_ERR_INVALID_ARG, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(VX_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < L.total) return fail(VX_ERR_WORKSPACE, "workspace smaller than vx_workspace_bytes()");
    return VX_OK;
}

// Argument checks shared by the chunk calls (vx_plot_chunk,
// vx_plot_staged_chunk).
vx_status check_chunk_args(uint32_t chunk_bits, uint32_t chunk, uint64_t t1_capacity, const vx_plot_buffers *b,
                           const uint64_t *d_t1_count) {
    if (chunk_bits > kMaxChunkBits || chunk >= (1u << chunk_bits))
        return fail(VX_ERR_INVALID_ARG, "chunk_bits must be at most 8 and chunk below 2^chunk_bits");
    if (t1_capacity == 0 || t1_capacity >= (1ull << 32))
        return fail(VX_ERR_INVALID_ARG, "t1_capacity must be in [1, 2^32)");
    if (!b || !d_t1_count) return fail(VX_ERR_INVALID_ARG, "buffers or d_t1_count is NULL");
    if (!b->t1_keys || !b->t1_nonces || !b->bucket_offsets || !b->t2_count || (b->t2_capacity && !b->t2))
        return fail(VX_ERR_INVALID_ARG, "NULL buffer");
    if (!aligned(b->t1_keys, 8) || !aligned(b->t1_nonces, 4) || !aligned(b->bucket_offsets, 4) ||
        !aligned(b->t2_count, 8) || !aligned(d_t1_count, 8) || (b->t2 && !aligned(b->t2, 16)))
        return fail(VX_ERR_INVALID_ARG, "misaligned buffer");
    return VX_OK;
}

// Stores a chunk's record count m (known on the host) in *d_t1_count and
// checks it against the capacity; an empty chunk's outputs are written here
// (*empty = true: nothing is left to do).
vx_status publish_chunk_count(uint64_t m, uint64_t *d_t1_count, uint64_t t1_capacity, const vx_plot_buffers *b,
                              hipStream_t s, bool *empty) {
    *empty = false;
    VX_HIP(hipMemcpyAsync(d_t1_count, &m, sizeof(m), hipMemcpyHostToDevice, s), "chunk count");
    VX_HIP(hipStreamSynchronize(s), "chunk count");  // m lives on this stack frame
    if (m > t1_capacity) return fail(VX_ERR_WORKSPACE, "the chunk holds more records than t1_capacity");
    if (m == 0) {
        VX_HIP(vxk::launch_fill_u32(b->bucket_offsets, (uint64_t)VX_NUM_BUCKETS + 1, 0u, s), "empty chunk");
        VX_HIP(vxk::launch_zero_u64(b->t2_count, 1, s), "empty chunk");
        *empty = true;
    }
    return VX_OK;
}

// Offsets of the buckets outside chunk `chunk`: 0 before it, m after it
// (and at the end).
vx_status fill_outside_offsets(uint32_t *offsets, uint32_t chunk_bits, uint32_t chunk, uint64_t m, hipStream_t s) {
    const uint64_t b0 = (uint64_t)chunk << (VX_BUCKET_BITS - chunk_bits);
    const uint64_t b1 = (uint64_t)(chunk + 1) << (VX_BUCKET_BITS - chunk_bits);
    if (b0) VX_HIP(vxk::launch_fill_u32(offsets, b0, 0u, s), "chunk offsets");
    VX_HIP(vxk::launch_fill_u32(offsets + b1, (uint64_t)VX_NUM_BUCKETS + 1 - b1, (uint32_t)m, s), "chunk offsets");
    return VX_OK;
}

}  // namespace

extern "C" {

uint64_t vx_default_threshold(uint32_t k) {
    if (k < 1 || k > 63) return 0;
    return 1ull << (64 - k);
}

size_t vx_workspace_bytes(const vx_plot_params *params, int which_call, const vx_tuning *tuning) {
    Plan P;
    if (which_call < VX_CALL_BUCKET_SORT || which_call > VX_CALL_PLOT) return 0;
    if (make_plan(params, tuning, &P) != VX_OK) return 0;
    return layout(P, which_call).total;
}

uint32_t vx_partition_passes(const vx_plot_params *params, const vx_tuning *tuning) {
    Plan P;
    if (make_plan(params, tuning, &P) != VX_OK) return 0;
    return P.npass;
}

uint32_t vx_hash_slices(const vx_plot_params *params, const vx_tuning *tuning) {
    Plan P;
    if (make_plan(params, tuning, &P) != VX_OK) return 0;
    return P.hq;
}

uint32_t vx_front_passes(const vx_plot_params *params, const vx_tuning *tuning) {
    Plan P;
    if (make_plan(params, tuning, &P) != VX_OK) return 0;
    return hash_passes(P);
}

uint32_t vx_tail_slices(const vx_plot_params *params, const vx_tuning *tuning) {
    Plan P;
    if (make_plan(params, tuning, &P) != VX_OK) return 0;
    return P.zt;
}

uint64_t vx_t2_capacity_hint(uint32_t k, uint64_t threshold) {
    if (k < 1 || k > 31) return 0;
    // Expected pairs per record for uniform keys: neighbours within T inside
    // the record's bucket.  With lambda = 2^(k-24) records per bucket and
    // bucket width W = 2^40, a record sees on average lambda * min(T, W) / W
    // later neighbours within T (at most lambda / 2 counting all pairs once).
    const double n = (double)(1ull << k);
    const double lam = n / (double)VX_NUM_BUCKETS;
    const double w = (double)(1ull << 40);
    const double t = threshold >= (1ull << 40) ? w : (double)threshold;
    double per = lam * (t / w) * (1.0 - 0.5 * t / w);
    double expect = n * per;
    double cap = expect * 1.05 + 8.0 * __builtin_sqrt(expect + 1.0) + 4096.0;
    return (uint64_t)cap;
}

const char *vx_last_error(void) { return g_err; }

vx_status vx_hash_table1(const vx_plot_params *params, uint64_t *d_keys, void *stream) {
    Plan P;
    vx_status st = make_plan(params, nullptr, &P);
    if (st != VX_OK) return st;
    if (!d_keys || !aligned(d_keys, 8)) return fail(VX_ERR_INVALID_ARG, "d_keys must be 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    VX_HIP(vxk::launch_hash_table1(P.key_words, P.n, P.W, P.chunk1, d_keys, nullptr, 0, s), "hash");
    g_err[0] = 0;
    return VX_OK;
}

vx_status vx_bucket_sort(const vx_plot_params *params, const uint64_t *d_keys, uint64_t *d_t1_keys,
                         uint32_t *d_t1_nonces, uint32_t *d_offsets, void *d_workspace,
                         size_t workspace_bytes, const vx_tuning *tuning, void *stream) {
    Plan P;
    vx_status st = make_plan(params, tuning, &P);
    if (st != VX_OK) return st;
    P.hs = false;  // caller keys: the first pass runs on them
    if (!d_keys || !d_t1_keys || !d_t1_nonces || !d_offsets)
        return fail(VX_ERR_INVALID_ARG, "NULL buffer");
    if (!aligned(d_keys, 8) || !aligned(d_t1_keys, 8) || !aligned(d_t1_nonces, 4) || !aligned(d_offsets, 4))
        return fail(VX_ERR_INVALID_ARG, "misaligned buffer");
    Layout L = layout(P, VX_CALL_BUCKET_SORT);
    if ((st = check_ws(L, d_workspace, workspace_bytes)) != VX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    VX_HIP(vxk::launch_reset(at<uint32_t>(d_workspace, L.header), kHeaderWords, s), "reset");
    st = run_partition(P, L, d_workspace, d_keys, false, d_t1_keys, d_t1_nonces, P.npass, s, nullptr);
    if (st == VX_OK)
        st = run_group_sort(P, L, d_workspace, d_t1_keys, d_t1_nonces, d_offsets, nullptr, 0, 1u << P.G, 0, s);
    if (st == VX_OK) g_err[0] = 0;
    return st;
}

vx_status vx_match_table2(const vx_plot_params *params, const uint64_t *d_t1_keys,
                          const uint32_t *d_t1_nonces, const uint32_t *d_offsets, vx_t2_record *d_t2,
                          uint64_t t2_capacity, uint64_t *d_t2_count, void *d_workspace,
                          size_t workspace_bytes, const vx_tuning *tuning, void *stream) {
    Plan P;
    vx_status st = make_plan(params, tuning, &P);
    if (st != VX_OK) return st;
    if (!d_t1_keys || !d_t1_nonces || !d_offsets || !d_t2_count || (t2_capacity && !d_t2))
        return fail(VX_ERR_INVALID_ARG, "NULL buffer");
    if (!aligned(d_t1_keys, 8) || !aligned(d_t2_count, 8) || (d_t2 && !aligned(d_t2, 16)))
        return fail(VX_ERR_INVALID_ARG, "misaligned buffer");
    Layout L = layout(P, VX_CALL_MATCH);
    if ((st = check_ws(L, d_workspace, workspace_bytes)) != VX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    (void)d_offsets;  // validated above; the match walks Table 1 itself
    VX_HIP(vxk::launch_reset(at<uint32_t>(d_workspace, L.header), kHeaderWords, s), "reset");
    VX_HIP(vxk::launch_match_count(d_t1_keys, (uint32_t)P.n, P.cb, P.T, at<uint64_t>(d_workspace, L.mcount),
                                   at<uint8_t>(d_workspace, L.pcnt), s),
           "match count");
    st = run_match(P, L, d_workspace, d_t1_keys, d_t1_nonces, d_t2, t2_capacity, d_t2_count, nullptr, nullptr, 1,
                   0, 0, s, nullptr, true);
    if (st == VX_OK) g_err[0] = 0;
    return st;
}

uint64_t vx_chunk_capacity_hint(uint32_t k, uint32_t chunk_bits, uint64_t threshold, uint64_t *t2_capacity) {
    if (t2_capacity) *t2_capacity = 0;
    if (k < 1 || k > 32 || chunk_bits > kMaxChunkBits || chunk_bits > k) return 0;
    const double recs = __builtin_ldexp(1.0, (int)k - (int)chunk_bits);
    const double cap1 = recs + 8.0 * __builtin_sqrt(recs) + 4096.0;
    if (cap1 >= 4294967296.0) return 0;  // a chunk holds fewer than 2^32 records
    if (t2_capacity) {
        // As vx_t2_capacity_hint, for the chunk's share of the records.
        const double lam = __builtin_ldexp(1.0, (int)k - 24);
        const double w = (double)(1ull << 40);
        const double t = threshold >= (1ull << 40) ? w : (double)threshold;
        const double expect = recs * lam * (t / w) * (1.0 - 0.5 * t / w);
        *t2_capacity = (uint64_t)(expect * 1.05 + 8.0 * __builtin_sqrt(expect + 1.0) + 4096.0);
    }
    return (uint64_t)cap1;
}

size_t vx_chunk_workspace_bytes(const vx_plot_params *params, uint32_t chunk_bits, uint64_t t1_capacity,
                                const vx_tuning *tuning) {
    Plan P;
    if (chunk_bits > kMaxChunkBits || t1_capacity == 0 || t1_capacity >= (1ull << 32)) return 0;
    if (make_plan(params, tuning, &P, t1_capacity, 32) != VX_OK) return 0;
    if (P.fused) return 0;
    return layout(P, kCallChunk).total;
}

vx_status vx_plot_chunk(const vx_plot_params *params, uint32_t chunk_bits, uint32_t chunk,
                        const vx_plot_buffers *b, uint64_t t1_capacity, uint64_t *d_t1_count,
                        const vx_tuning *tuning, void *stream) {
    Plan Pc;
    vx_status st = make_plan(params, tuning, &Pc, t1_capacity ? t1_capacity : 1, 32);
    if (st != VX_OK) return st;
    if ((st = check_chunk_args(chunk_bits, chunk, t1_capacity, b, d_t1_count)) != VX_OK) return st;
    if (Pc.fused) return fail(VX_ERR_UNSUPPORTED, "chunked plots use the split sort and match");
    Layout L = layout(Pc, kCallChunk);
    if ((st = check_ws(L, b->workspace, b->workspace_bytes)) != VX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    void *ws = b->workspace;
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    uint64_t *keys_in = at<uint64_t>(ws, L.keys_no);
    uint32_t *nonces_in = at<uint32_t>(ws, L.nonces_in);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(hdr + kHdrChunkCount);
    VX_HIP(vxk::launch_reset(hdr, kHeaderWords, s), "reset");
    // Hash every nonce of the plot and keep this chunk's bucket range.
    const uint64_t n_all = 1ull << params->k;
    const uint32_t tiles = clampu((int64_t)(n_all >> 16), 1, 16384);
    VX_HIP(vxk::launch_hash_filter(Pc.key_words, n_all, tiles, (n_all + tiles - 1) / tiles, chunk_bits, chunk,
                                   keys_in, nonces_in, t1_capacity, count, s),
           "chunk hash");
    // The sort is planned for the records kept: wait for their number.
    uint64_t m = 0;
    VX_HIP(hipMemcpyAsync(&m, count, sizeof(m), hipMemcpyDeviceToHost, s), "chunk count");
    VX_HIP(hipStreamSynchronize(s), "chunk count");
    bool empty = false;
    if ((st = publish_chunk_count(m, d_t1_count, t1_capacity, b, s, &empty)) != VX_OK) return st;
    if (empty) {
        g_err[0] = 0;
        return VX_OK;
    }
    Plan P;
    if ((st = make_plan(params, tuning, &P, m, 32)) != VX_OK) return st;
    // Same groups and digits as the capacity plan, so L fits (it was sized
    // for t1_capacity >= m records).
    st = run_partition(P, L, ws, keys_in, false, b->t1_keys, b->t1_nonces, P.npass, s, nullptr, nonces_in);
    if (st != VX_OK) return st;
    // Only the chunk's groups hold records (when the groups are at least as
    // fine as the chunks): sort those, and fill the other buckets' offsets.
    const bool own = chunk_bits <= P.G;
    const uint32_t g0 = own ? chunk << (P.G - chunk_bits) : 0;
    const uint32_t gn = own ? 1u << (P.G - chunk_bits) : 1u << P.G;
    st = run_group_sort(P, L, ws, b->t1_keys, b->t1_nonces, b->bucket_offsets, at<uint8_t>(ws, L.pcnt), g0, gn, 0,
                        s);
    if (st == VX_OK && own) st = fill_outside_offsets(b->bucket_offsets, chunk_bits, chunk, m, s);
    if (st == VX_OK)
        st = run_match(P, L, ws, b->t1_keys, b->t1_nonces, b->t2, b->t2_capacity, b->t2_count, nullptr, nullptr, 1,
                       0, 0, s);
    if (st == VX_OK) g_err[0] = 0;
    return st;
}

size_t vx_stage_bytes(const vx_plot_params *params, uint32_t chunk_bits, const vx_tuning *tuning) {
    Plan P;
    if (chunk_bits > kMaxChunkBits) return 0;
    if (make_plan(params, tuning, &P, 0, 32, (int)chunk_bits) != VX_OK) return 0;
    return stage_layout(P).total;
}

vx_status vx_stage_plot(const vx_plot_params *params, uint32_t chunk_bits, const vx_tuning *tuning, void *d_stage,
                        size_t stage_bytes, void *stream) {
    if (chunk_bits > kMaxChunkBits) return fail(VX_ERR_INVALID_ARG, "chunk_bits must be at most 8");
    Plan P;
    vx_status st = make_plan(params, tuning, &P, 0, 32, (int)chunk_bits);
    if (st != VX_OK) return st;
    if (!d_stage) return fail(VX_ERR_INVALID_ARG, "stage is NULL");
    if (!aligned(d_stage, 256)) return fail(VX_ERR_INVALID_ARG, "misaligned stage");
    const StageLayout S = stage_layout(P);
    if (stage_bytes < S.total) return fail(VX_ERR_WORKSPACE, "stage smaller than vx_stage_bytes");
    hipStream_t s = (hipStream_t)stream;
    uint32_t *hdr = at<uint32_t>(d_stage, S.header);
    uint32_t id[kStageIdWords];
    stage_id(P, chunk_bits, id);
    VX_HIP(vxk::launch_reset(hdr, kHeaderWords, s), "reset");
    VX_HIP(vxk::launch_put_words(hdr + 1, id + 1, kStageIdWords - 1, s), "stage header");
    if (P.deep) {
        st = stage_sliced_front(P, S, chunk_bits, d_stage, s);
        if (st == VX_OK) g_err[0] = 0;
        return st;
    }
    VX_HIP(vxk::launch_fill_u32(at<uint32_t>(d_stage, S.fill), 1ull << P.D[0], 0u, s), "reset");
    VX_HIP(vxk::launch_hash_scatter(P.key_words, P.n, P.D[0], P.R[0], at<uint64_t>(d_stage, S.keys),
                                    at<uint32_t>(d_stage, S.nonces), at<uint32_t>(d_stage, S.fill), hdr + kHdrStatus,
                                    s),
           "stage hash");
    g_err[0] = 0;
    return VX_OK;
}

size_t vx_staged_chunk_workspace_bytes(const vx_plot_params *params, uint32_t chunk_bits, uint64_t t1_capacity,
                                       const vx_tuning *tuning) {
    Plan P;
    if (chunk_bits > kMaxChunkBits || t1_capacity == 0 || t1_capacity >= (1ull << 32)) return 0;
    if (make_plan(params, tuning, &P, t1_capacity, 32, (int)chunk_bits) != VX_OK) return 0;
    return layout(P, kCallStagedChunk).total;
}

}  // extern "C"

namespace {
// Chunk `chunk` of a stage that holds the third pass's regions (P.deep):
// the chunk's second-pass group starts (summed over the slices' own
// regions), then its third-pass region bounds and group starts, from a copy
// of its fills (the stage stays read-only), the group sort straight from
// the stage, and the match.
vx_status staged_chunk_sorted(const Plan &Pc, const Layout &L, const StageLayout &S, uint32_t cb, uint32_t chunk,
                              const void *d_stage, const vx_plot_buffers *b, uint64_t t1_capacity,
                              uint64_t *d_t1_count, hipStream_t s) {
    void *ws = b->workspace;
    void *stage = const_cast<void *>(d_stage);
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    const uint32_t b01 = Pc.D[0] + Pc.D[1], D2 = Pc.D[2];
    const uint32_t nd01c = 1u << (b01 - cb), first01 = chunk * nd01c;
    const uint32_t g_first = first01 << D2, ng = nd01c << D2;
    uint32_t *gst1 = at<uint32_t>(ws, L.gstart[1]);
    VX_HIP(vxk::launch_reset(hdr, kHeaderWords, s), "reset");
    VX_HIP(vxk::launch_region_scan_slices(at<uint32_t>(stage, S.fill1) + first01, Pc.hq, 1u << b01, nd01c,
                                          Pc.R[1], gst1 + first01, s),
           "chunk regions");
    uint32_t m32 = 0, id[kStageIdWords], want[kStageIdWords];
    VX_HIP(hipMemcpyAsync(&m32, gst1 + first01 + nd01c, sizeof(m32), hipMemcpyDeviceToHost, s), "chunk count");
    VX_HIP(hipMemcpyAsync(id, at<const uint32_t>(stage, S.header), sizeof(id), hipMemcpyDeviceToHost, s),
           "stage header");
    VX_HIP(hipStreamSynchronize(s), "chunk count");
    stage_id(Pc, cb, want);
    if (memcmp(id + 1, want + 1, (kStageIdWords - 1) * 4) != 0)
        return fail(VX_ERR_INVALID_ARG, "the stage was made for another key, k, chunk_bits or tuning");
    const uint64_t m = m32;
    bool empty = false;
    vx_status st = publish_chunk_count(m, d_t1_count, t1_capacity, b, s, &empty);
    if (st != VX_OK) return st;
    if (empty) {
        g_err[0] = 0;
        return VX_OK;
    }
    Plan P = Pc;  // the stage's digits and regions, the chunk's records
    P.n = m;
    uint32_t *fill2 = at<uint32_t>(ws, L.fill[2]) + g_first;
    VX_HIP(hipMemcpyAsync(fill2, at<const uint32_t>(stage, S.fill) + g_first, (size_t)ng * 4,
                          hipMemcpyDeviceToDevice, s),
           "chunk fills");
    VX_HIP(vxk::launch_region_bounds(fill2, 0, ng, P.R[2], at<uint32_t>(ws, L.seg_lo[2]) + g_first,
                                     at<uint32_t>(ws, L.seg_hi[2]) + g_first, s),
           "chunk regions");
    VX_HIP(vxk::launch_colscan(fill2, at<uint32_t>(ws, L.off[2]) + g_first, nd01c, 1, 1u << D2, gst1 + first01,
                               at<uint32_t>(ws, L.gstart[2]) + g_first, ng, (uint32_t)m, s),
           "chunk scan");
    const uint64_t creg = (uint64_t)P.R[2] << (P.G - cb);
    st = run_group_sort(P, L, ws, b->t1_keys, b->t1_nonces, b->bucket_offsets, at<uint8_t>(ws, L.pcnt), g_first, ng,
                        0, s, false, at<const uint64_t>(stage, S.keys) + chunk * creg,
                        at<const uint32_t>(stage, S.nonces) + chunk * creg);
    if (st != VX_OK) return st;
    if ((st = fill_outside_offsets(b->bucket_offsets, cb, chunk, m, s)) != VX_OK) return st;
    st = run_match(P, L, ws, b->t1_keys, b->t1_nonces, b->t2, b->t2_capacity, b->t2_count, nullptr, nullptr, 1, 0,
                   0, s);
    if (st == VX_OK) g_err[0] = 0;
    return st;
}
}  // namespace

extern "C" {

vx_status vx_plot_staged_chunk(const vx_plot_params *params, uint32_t chunk_bits, uint32_t chunk,
                               const void *d_stage, size_t stage_bytes, const vx_plot_buffers *b,
                               uint64_t t1_capacity, uint64_t *d_t1_count, const vx_tuning *tuning, void *stream) {
    vx_status st = check_chunk_args(chunk_bits, chunk, t1_capacity, b, d_t1_count);
    if (st != VX_OK) return st;
    Plan Pc;
    if ((st = make_plan(params, tuning, &Pc, t1_capacity, 32, (int)chunk_bits)) != VX_OK) return st;
    if (!d_stage) return fail(VX_ERR_INVALID_ARG, "stage is NULL");
    if (!aligned(d_stage, 256)) return fail(VX_ERR_INVALID_ARG, "misaligned stage");
    const Layout L = layout(Pc, kCallStagedChunk);
    if ((st = check_ws(L, b->workspace, b->workspace_bytes)) != VX_OK) return st;
    const StageLayout S = stage_layout(Pc);
    if (stage_bytes < S.total) return fail(VX_ERR_INVALID_ARG, "stage smaller than these parameters need");
    hipStream_t s = (hipStream_t)stream;
    void *ws = b->workspace;
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    if (Pc.deep) return staged_chunk_sorted(Pc, L, S, chunk_bits, chunk, d_stage, b, t1_capacity, d_t1_count, s);
    // The chunk's first-pass regions in the stage, and where it starts.
    const uint32_t ndc = 1u << (Pc.D[0] - chunk_bits);
    const uint32_t d_first = chunk * ndc;
    const uint64_t *stage_k = at<const uint64_t>(const_cast<void *>(d_stage), S.keys) + (uint64_t)d_first * Pc.R[0];
    const uint32_t *stage_n = at<const uint32_t>(const_cast<void *>(d_stage), S.nonces) + (uint64_t)d_first * Pc.R[0];
    const uint32_t *stage_fill = at<const uint32_t>(const_cast<void *>(d_stage), S.fill) + d_first;
    VX_HIP(vxk::launch_reset(hdr, kHeaderWords, s), "reset");
    for (uint32_t i = 1; i < Pc.npass; ++i)
        VX_HIP(vxk::launch_fill_u32(at<uint32_t>(ws, L.fill[i]), 1ull << (Pc.pre[i] + Pc.D[i]), 0u, s), "reset");
    uint32_t *gst0 = at<uint32_t>(ws, L.gstart[0]);
    VX_HIP(vxk::launch_region_scan(stage_fill, ndc, Pc.R[0], at<uint32_t>(ws, L.seg_lo[0]) + d_first,
                                   at<uint32_t>(ws, L.seg_hi[0]) + d_first, gst0 + d_first, s),
           "chunk regions");
    // The sort is planned for the chunk's records: wait for their number,
    // and check that the stage was made for these parameters.
    uint32_t m32 = 0, id[kStageIdWords], want[kStageIdWords];
    VX_HIP(hipMemcpyAsync(&m32, gst0 + d_first + ndc, sizeof(m32), hipMemcpyDeviceToHost, s), "chunk count");
    VX_HIP(hipMemcpyAsync(id, at<const uint32_t>(const_cast<void *>(d_stage), S.header), sizeof(id),
                          hipMemcpyDeviceToHost, s),
           "stage header");
    VX_HIP(hipStreamSynchronize(s), "chunk count");
    stage_id(Pc, chunk_bits, want);
    if (memcmp(id + 1, want + 1, (kStageIdWords - 1) * 4) != 0)
        return fail(VX_ERR_INVALID_ARG, "the stage was made for another key, k, chunk_bits or tuning");
    const uint64_t m = m32;
    bool empty = false;
    if ((st = publish_chunk_count(m, d_t1_count, t1_capacity, b, s, &empty)) != VX_OK) return st;
    if (empty) {
        g_err[0] = 0;
        return VX_OK;
    }
    Plan P;
    if ((st = make_plan(params, tuning, &P, m, 32, (int)chunk_bits)) != VX_OK) return st;
    // Same digits and regions as the capacity plan, so L fits.  Pass 1 reads
    // the stage; later passes alternate between the workspace's buffers.
    for (uint32_t i = 1; i < P.npass; ++i) {
        PassBufs B = pass_bufs(P, L, ws, nullptr, b->t1_keys, b->t1_nonces, i);
        if (i == 1) {
            B.in_k = stage_k;
            B.in_n = stage_n;
        }
        const uint32_t sh = P.pre[i] - P.D[0];
        if ((st = run_pass(P, L, ws, B, i, d_first << sh, (d_first + ndc) << sh, s, d_first << sh)) != VX_OK)
            return st;
    }
    const uint32_t gsh = P.G - P.D[0];
    st = run_group_sort(P, L, ws, b->t1_keys, b->t1_nonces, b->bucket_offsets, at<uint8_t>(ws, L.pcnt),
                        d_first << gsh, ndc << gsh, 0, s);
    if (st != VX_OK) return st;
    // Buckets before the chunk start at 0, those after it (and the end) at m.
    if ((st = fill_outside_offsets(b->bucket_offsets, chunk_bits, chunk, m, s)) != VX_OK) return st;
    st = run_match(P, L, ws, b->t1_keys, b->t1_nonces, b->t2, b->t2_capacity, b->t2_count, nullptr, nullptr, 1, 0,
                   0, s);
    if (st == VX_OK) g_err[0] = 0;
    return st;
}

}  // extern "C"

namespace vxs {
void set_error(const char *msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }
}  // namespace vxs

namespace {

// Internal streams for vx_plot_batch, created once per device at default
// priority, with the events that fork from and join into the caller's
// stream.  The mutex serialises enqueuing from different host threads.
constexpr int kBatchLanes = 4;

struct Lanes {
    std::mutex mu;
    bool ready = false;
    hipStream_t s[kBatchLanes] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kBatchLanes] = {};
};

Lanes g_lanes[kMaxDevices];
std::mutex g_lanes_mu;

vx_status lanes_for_current_device(Lanes **out) {
    int dev = 0;
    VX_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(VX_ERR_UNSUPPORTED, "device index out of range");
    Lanes &L = g_lanes[dev];
    std::lock_guard<std::mutex> guard(g_lanes_mu);
    if (!L.ready) {
        for (int l = 0; l < kBatchLanes; ++l) {
            VX_HIP(hipStreamCreateWithFlags(&L.s[l], hipStreamNonBlocking), "batch stream");
            VX_HIP(hipEventCreateWithFlags(&L.join[l], hipEventDisableTiming), "batch event");
        }
        VX_HIP(hipEventCreateWithFlags(&L.fork, hipEventDisableTiming), "batch event");
        L.ready = true;
    }
    *out = &L;
    return VX_OK;
}

// Every check of a whole plot's arguments (vx_plot, and each plot of
// vx_plot_batch before anything is enqueued); fills the plan and layout.
vx_status check_plot(const vx_plot_params *params, const vx_plot_buffers *b, const vx_tuning *tuning, Plan *P,
                     Layout *L) {
    vx_status st = make_plan(params, tuning, P);
    if (st != VX_OK) return st;
    if (!b) return fail(VX_ERR_INVALID_ARG, "buffers is NULL");
    if (!b->t1_keys || !b->t1_nonces || !b->bucket_offsets || !b->t2_count || (b->t2_capacity && !b->t2))
        return fail(VX_ERR_INVALID_ARG, "NULL buffer");
    if (!aligned(b->t1_keys, 8) || !aligned(b->t1_nonces, 4) || !aligned(b->bucket_offsets, 4) ||
        !aligned(b->t2_count, 8) || (b->t2 && !aligned(b->t2, 16)))
        return fail(VX_ERR_INVALID_ARG, "misaligned buffer");
    *L = layout(*P, VX_CALL_PLOT);
    return check_ws(*L, b->workspace, b->workspace_bytes);
}

// pipelined: the plan's slices may run on a second stream (vx_plot); batch
// lanes run every plot on its lane alone, and keep the workspace's status
// word (cleared once per workspace by vx_plot_batch), so that it collects
// the status of every plot that used the workspace.
// The header words (the status word too, unless keep_status) and the
// region fill counts of a plot, cleared before its first kernel.
vx_status plot_reset(const Plan &P, const Layout &L, void *ws, bool keep_status, hipStream_t s) {
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    static_assert(kHdrStatus == 0, "the status word leads the header");
    if (keep_status)
        VX_HIP(vxk::launch_reset(hdr + 1, kHeaderWords - 1, s), "reset");
    else
        VX_HIP(vxk::launch_reset(hdr, kHeaderWords, s), "reset");
    for (uint32_t i = 0; P.hs && i < P.npass; ++i)
        VX_HIP(vxk::launch_fill_u32(at<uint32_t>(ws, L.fill[i]),
                                    i == 0 ? (uint64_t)front_fill_stride(P) * P.hq
                                           : (uint64_t)(i == 1 && P.deep ? P.hq : 1) << (P.pre[i] + P.D[i]),
                                    0u,
                                    s),
               "reset");
    return VX_OK;
}

vx_status plot_tail(const Plan &P, const Layout &L, const vx_plot_buffers *b, hipEvent_t *ev, hipStream_t s,
                    bool pipelined, uint32_t front_passes);

vx_status plot_impl(const vx_plot_params *params, const vx_plot_buffers *b, const vx_tuning *tuning,
                    hipEvent_t *ev, void *stream, bool pipelined, bool keep_status = false) {
    Plan P;
    Layout L;
    vx_status st = check_plot(params, b, tuning, &P, &L);
    if (st != VX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    void *ws = b->workspace;
    uint64_t *keys_no = at<uint64_t>(ws, L.keys_no);
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    if ((st = plot_reset(P, L, ws, keep_status, s)) != VX_OK) return st;
    VX_HIP(mark(ev, 0, s), "event");
    if (P.hs && P.hq > 1) {
        st = run_sliced_front(P, L, ws, s, ev);
        if (st != VX_OK) return st;
    } else if (P.hs) {
        // Hash + first partition pass in one kernel, then the regions' bounds.
        VX_HIP(vxk::launch_hash_scatter(P.key_words, P.n, P.D[0], P.R[0], keys_no, at<uint32_t>(ws, L.reg_nonces),
                                        at<uint32_t>(ws, L.fill[0]), hdr + kHdrStatus, s),
               "hash + first pass");
        VX_HIP(mark(ev, 1, s), "event");
        VX_HIP(vxk::launch_region_scan(at<uint32_t>(ws, L.fill[0]), 1u << P.D[0], P.R[0],
                                       at<uint32_t>(ws, L.seg_lo[0]), at<uint32_t>(ws, L.seg_hi[0]),
                                       at<uint32_t>(ws, L.gstart[0]), s),
               "region scan");
        VX_HIP(mark(ev, 2, s), "event");
    } else {
        VX_HIP(vxk::launch_hash_table1(P.key_words, P.n, P.W, P.chunk1, keys_no, at<uint32_t>(ws, L.hist[0]),
                                       P.D[0], s),
               "hash");
        VX_HIP(mark(ev, 1, s), "event");
    }
    st = plot_tail(P, L, b, ev, s, pipelined, hash_passes(P));
    if (st == VX_OK) g_err[0] = 0;
    return st;
}

// Everything after the hash (and the passes it files): the remaining
// partition passes, the sort, the match and Table-2 hash.
vx_status plot_tail(const Plan &P, const Layout &L, const vx_plot_buffers *b, hipEvent_t *ev, hipStream_t s,
                    bool pipelined, uint32_t front_passes) {
    vx_status st = VX_OK;
    void *ws = b->workspace;
    uint64_t *keys_no = at<uint64_t>(ws, L.keys_no);
    uint32_t *hdr = at<uint32_t>(ws, L.header);
    if (!P.fused && pipelined && P.slices > 1) {
        st = run_partition(P, L, ws, keys_no, true, b->t1_keys, b->t1_nonces, 1, s, ev, nullptr, front_passes);
        if (st == VX_OK) st = run_pipelined(P, L, ws, b, keys_no, s, ev);
    } else if (!P.fused && P.zt > 1) {
        // Passes before the third as separate kernels, then the pipelined tail.
        st = run_partition(P, L, ws, keys_no, true, b->t1_keys, b->t1_nonces, std::min(P.npass, 2u), s, ev, nullptr,
                           front_passes);
        if (st != VX_OK) return st;
        VX_HIP(mark(ev, 4, s), "event");
        VX_HIP(mark(ev, 5, s), "event");
        st = run_pipe_tail(P, L, ws, b, s);
        if (st != VX_OK) return st;
        VX_HIP(mark(ev, 6, s), "event");
    } else if (!P.fused) {
        // Separate kernels: the sort stores each record's pair count while
        // the groups are in LDS, then the match kernel reads nonces and counts.
        st = run_partition(P, L, ws, keys_no, true, b->t1_keys, b->t1_nonces, P.npass, s, ev, nullptr, front_passes);
        if (st != VX_OK) return st;
        st = run_group_sort(P, L, ws, b->t1_keys, b->t1_nonces, b->bucket_offsets, at<uint8_t>(ws, L.pcnt), 0,
                            1u << P.G, 0, s);
        if (st != VX_OK) return st;
        VX_HIP(mark(ev, 4, s), "event");
        st = run_match(P, L, ws, b->t1_keys, b->t1_nonces, b->t2, b->t2_capacity, b->t2_count, nullptr, nullptr,
                       1, 0, 0, s, ev);
    } else {
        st = run_partition(P, L, ws, keys_no, true, b->t1_keys, b->t1_nonces, P.npass, s, ev, nullptr, front_passes);
        if (st != VX_OK) return st;
        uint64_t *words = at<uint64_t>(ws, L.lbwords);
        VX_HIP(vxk::launch_zero_u64(words, 1u << P.G, s), "zero look-back words");
        VX_HIP(mark(ev, 4, s), "event");
        VX_HIP(mark(ev, 5, s), "event");
        const uint32_t last = P.npass - 1;
        const uint64_t *in_k = nullptr;
        const uint32_t *in_n = nullptr, *in_lo = nullptr, *in_hi = nullptr;
        if (P.hs) {
            const PassBufs B = pass_bufs(P, L, ws, nullptr, b->t1_keys, b->t1_nonces, last);
            in_k = B.out_k;
            in_n = B.out_n;
            in_lo = at<uint32_t>(ws, L.seg_lo[last]);
            in_hi = at<uint32_t>(ws, L.seg_hi[last]);
        }
        VX_HIP(vxk::launch_group_match(P.key_words, b->t1_keys, b->t1_nonces, in_k, in_n, in_lo, in_hi,
                                       at<uint64_t>(ws, L.scr_keys), at<uint32_t>(ws, L.scr_nonces),
                                       at<uint32_t>(ws, L.gstart[last]), P.G, P.cap, b->bucket_offsets,
                                       (uint32_t)P.n, P.T, hdr + kHdrFusedTicket, words, hdr + kHdrStatus, b->t2,
                                       b->t2_capacity, b->t2_count, kLookbackSpinLimit, s),
               "sort + match");
        VX_HIP(mark(ev, 6, s), "event");
    }
    return st;
}

}  // namespace

extern "C" {

vx_status vx_plot(const vx_plot_params *params, const vx_plot_buffers *b, const vx_tuning *tuning,
                  void *stream) {
    return plot_impl(params, b, tuning, nullptr, stream, true);
}

vx_status vx_plot_with_events(const vx_plot_params *params, const vx_plot_buffers *b,
                              const vx_tuning *tuning, void *const *events, void *stream) {
    if (!events) return fail(VX_ERR_INVALID_ARG, "events is NULL");
    hipEvent_t ev[VX_PLOT_EVENTS];
    for (int i = 0; i < VX_PLOT_EVENTS; ++i) {
        if (!events[i]) return fail(VX_ERR_INVALID_ARG, "NULL event");
        ev[i] = (hipEvent_t)events[i];
    }
    return plot_impl(params, b, tuning, ev, stream, true);
}

vx_status vx_plot_batch(const vx_plot_params *params, const vx_plot_buffers *buffers, uint32_t n,
                        const vx_tuning *tuning, void *stream) {
    if (n && (!params || !buffers)) return fail(VX_ERR_INVALID_ARG, "NULL params or buffers");
    // Validate everything before enqueuing anything.
    std::vector<Plan> plan(n);
    std::vector<Layout> lay(n);
    for (uint32_t i = 0; i < n; ++i) {
        vx_status st = check_plot(&params[i], &buffers[i], tuning ? &tuning[i] : nullptr, &plan[i], &lay[i]);
        if (st != VX_OK) return st;
    }
    if (n == 0) return VX_OK;
    hipStream_t s = (hipStream_t)stream;
    Lanes *ln = nullptr;
    vx_status st = lanes_for_current_device(&ln);
    if (st != VX_OK) return st;
    // Plots that share a workspace form one chain (run in list order); chains
    // go, largest first, to the least loaded lane.
    std::vector<const void *> chain_ws;
    std::vector<uint64_t> chain_work;
    std::vector<std::vector<uint32_t>> chain_plots;
    for (uint32_t i = 0; i < n; ++i) {
        int c = -1;
        for (size_t j = 0; j < chain_ws.size(); ++j)
            if (chain_ws[j] == buffers[i].workspace) c = (int)j;
        if (c < 0) {
            c = (int)chain_ws.size();
            chain_ws.push_back(buffers[i].workspace);
            chain_work.push_back(0);
            chain_plots.emplace_back();
        }
        chain_plots[c].push_back(i);
        chain_work[c] += plan[i].n;
    }
    const size_t nchains = chain_ws.size();
    std::vector<int> order(nchains);
    for (size_t j = 0; j < nchains; ++j) order[j] = (int)j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return chain_work[x] > chain_work[y]; });
    std::vector<int> lane_of_chain(nchains, 0);
    uint64_t load[kBatchLanes] = {};
    for (int c : order) {
        int best = 0;
        for (int l = 1; l < kBatchLanes; ++l)
            if (load[l] < load[best]) best = l;
        lane_of_chain[c] = best;
        load[best] += chain_work[c];
    }
    size_t rounds = 0;
    for (auto &v : chain_plots) rounds = std::max(rounds, v.size());
    std::lock_guard<std::mutex> guard(ln->mu);
    // Every lane starts behind the work already on the caller's stream.
    VX_HIP(hipEventRecord(ln->fork, s), "batch fork");
    bool used[kBatchLanes] = {};
    for (size_t c = 0; c < nchains; ++c) used[lane_of_chain[c]] = true;
    for (int l = 0; l < kBatchLanes; ++l)
        if (used[l]) VX_HIP(hipStreamWaitEvent(ln->s[l], ln->fork, 0), "batch fork wait");
    // Each workspace's status word is cleared once, before its first plot;
    // the plots then leave it alone, so afterwards it holds the status bits
    // of every plot that used that workspace.
    auto clear_status = [&](uint32_t i, hipStream_t on) -> vx_status {
        VX_HIP(vxk::launch_reset(static_cast<uint32_t *>(buffers[i].workspace), 1, on), "batch status");
        return VX_OK;
    };
    // Round r takes the r-th plot of every chain (different workspaces).
    // Plots that ask for it (batch_shared_hash) and whose hash files two
    // passes share fused launches on the caller's stream (k_hash_pass over a
    // device work list): launch u hashes the
    // slices of unit u -- slices of one or more plots, large ones alone,
    // small ones packed up to 2^27 nonces -- while its other work-groups
    // file by the second digit the slices of unit u - 1 and, by the third,
    // parts of plots whose second pass is complete.  The third pass of a
    // plot needs all of its second, so only another plot's hash can hide it.
    // As soon as a plot's passes are done, its sort and match go to its
    // lane.  The other plots run whole on their lanes.
    std::vector<int> chain_of(n, -1);
    for (size_t c = 0; c < nchains; ++c)
        for (uint32_t i : chain_plots[c]) chain_of[i] = (int)c;
    auto hand_over = [&](uint32_t i, uint32_t passes_done) -> vx_status {
        const int l = lane_of_chain[chain_of[i]];
        VX_HIP(hipEventRecord(ln->fork, s), "batch hand-over");
        VX_HIP(hipStreamWaitEvent(ln->s[l], ln->fork, 0), "batch hand-over wait");
        return plot_tail(plan[i], lay[i], &buffers[i], nullptr, ln->s[l], false, passes_done);
    };
    for (size_t r = 0; r < rounds && st == VX_OK; ++r) {
        std::vector<uint32_t> F;
        for (size_t c = 0; c < nchains; ++c) {
            if (r >= chain_plots[c].size()) continue;
            const uint32_t i = chain_plots[c][r];
            const vx_tuning *ti = tuning ? &tuning[i] : nullptr;
            if (ti && ti->batch_shared_hash && front_fusable(plan[i])) {
                F.push_back(i);
                continue;
            }
            const hipStream_t lane = ln->s[lane_of_chain[c]];
            if (r == 0 && (st = clear_status(i, lane)) != VX_OK) break;
            if ((st = plot_impl(&params[i], &buffers[i], tuning ? &tuning[i] : nullptr, nullptr, lane, false, true)) !=
                VX_OK)
                break;
        }
        if (st != VX_OK || F.empty()) continue;
        // The caller's stream waits for the lanes of these plots' chains
        // (their previous plots' tails).
        if (r > 0)
            for (uint32_t i : F) {
                const int l = lane_of_chain[chain_of[i]];
                VX_HIP(hipEventRecord(ln->join[l], ln->s[l]), "batch round");
                VX_HIP(hipStreamWaitEvent(s, ln->join[l], 0), "batch round wait");
            }
        std::stable_sort(F.begin(), F.end(), [&](uint32_t x, uint32_t y) { return plan[x].n > plan[y].n; });
        for (uint32_t i : F) {
            if (r == 0 && (st = clear_status(i, s)) != VX_OK) break;
            if ((st = plot_reset(plan[i], lay[i], buffers[i].workspace, true, s)) != VX_OK) break;
        }
        if (st != VX_OK) break;
        // Units of slices (at most four, so that third-pass parts fit beside
        // the previous unit's second passes in one list).
        struct SliceRef {
            uint32_t plot, slice;
        };
        constexpr size_t kUnitMax = 4, kPartsPerPlot = 4;
        std::vector<std::vector<SliceRef>> units;
        uint64_t unit_nonces = 0;
        for (uint32_t i : F) {
            const Plan &P = plan[i];
            const uint64_t per_slice = (P.n + P.hq - 1) / P.hq;
            for (uint32_t q = 0; q < P.hq; ++q) {
                if (units.empty() || units.back().size() == kUnitMax ||
                    unit_nonces + per_slice > std::max<uint64_t>(1ull << 27, per_slice)) {
                    units.emplace_back();
                    unit_nonces = 0;
                }
                units.back().push_back({i, q});
                unit_nonces += per_slice;
            }
        }
        // Third-pass parts waiting for a launch, and how many of each plot's
        // are still to be filed.
        struct Part {
            uint32_t plot, a, e;  // the plot's second-pass regions [a, e)
        };
        std::vector<Part> pending;
        std::vector<uint32_t> parts_left(n, 0);
        const uint32_t U = (uint32_t)units.size();
        for (uint32_t u = 0; st == VX_OK && (u <= U || !pending.empty()); ++u) {
            vxk::HashPassList W;
            memset(&W, 0, sizeof(W));
            if (u < U)
                for (const SliceRef &x : units[u]) {
                    W.h[W.nh] = hash_slice(plan[x.plot], lay[x.plot], buffers[x.plot].workspace, x.slice);
                    W.h_items += W.h[W.nh++].items;
                }
            if (u >= 1 && u <= U)
                for (const SliceRef &x : units[u - 1]) {
                    W.p[W.np] = pass_slice(plan[x.plot], lay[x.plot], buffers[x.plot].workspace, x.slice);
                    W.p_items += W.p[W.np++].items;
                }
            std::vector<Part> taken;
            while (!pending.empty() && W.np < (uint32_t)vxk::kHashPassMaxSlices) {
                const Part pt = pending.front();
                pending.erase(pending.begin());
                const Plan &P = plan[pt.plot];
                const Layout &L = lay[pt.plot];
                void *ws = buffers[pt.plot].workspace;
                const PassBufs B2 = pass_bufs(P, L, ws, nullptr, buffers[pt.plot].t1_keys,
                                              buffers[pt.plot].t1_nonces, 2);
                vxk::PassSliceDesc &Q = W.p[W.np++];
                memset(&Q, 0, sizeof(Q));
                const uint32_t per = (P.R[1] + vxk::kHashScatterSub - 1) / vxk::kHashScatterSub;
                Q.keys = B2.in_k + (uint64_t)pt.a * P.R[1];
                Q.nonces = B2.in_n + (uint64_t)pt.a * P.R[1];
                Q.fill = at<uint32_t>(ws, L.fill[1]) + pt.a;
                Q.out_keys = B2.out_k;
                Q.out_nonces = B2.out_n;
                Q.out_fill = at<uint32_t>(ws, L.fill[2]);
                Q.status = at<uint32_t>(ws, L.header) + kHdrStatus;
                Q.R_in = P.R[1];
                Q.per = per;
                Q.shift = 64 - P.pre[2] - P.D[2];
                Q.bits = P.D[2];
                Q.R_out = P.R[2];
                Q.items = (pt.e - pt.a) * per;
                Q.r0 = pt.a;
                W.p_items += Q.items;
                taken.push_back(pt);
            }
            set_frac(W);
            // A zeroed ticket word: one of the batch words of one of the
            // round's plots' headers (a plot brings at most 16 slices and 4
            // third-pass parts, so the launches fit 21 words per plot).
            const uint32_t owner = F[u % F.size()];
            const uint32_t word = u / (uint32_t)F.size();
            if (word >= kBatchTicketWords) {
                st = fail(VX_ERR_UNSUPPORTED, "batch: too many fused launches in one round");
                break;
            }
            uint32_t *ticket = at<uint32_t>(buffers[owner].workspace, lay[owner].header) + kHdrBatchTicket + word;
            VX_HIP(vxk::launch_hash_pass(W, ticket, s), "batch hash");
            // Plots whose second pass finished in this launch: their group
            // starts, then (three passes) their third pass in later launches,
            // else their sort and match on their lane.
            if (u >= 1 && u <= U)
                for (const SliceRef &x : units[u - 1]) {
                    const uint32_t i = x.plot;
                    if (x.slice + 1 != plan[i].hq) continue;
                    if ((st = finish_front(plan[i], lay[i], buffers[i].workspace, s)) != VX_OK) break;
                    const Plan &P = plan[i];
                    if (P.npass == 3 && P.zt == 1 && P.D[2] <= (uint32_t)vxk::kHashPassMaxBits) {
                        const uint32_t N1 = 1u << (P.pre[1] + P.D[1]);
                        const uint32_t parts = (uint32_t)std::min<size_t>(kPartsPerPlot, N1);
                        for (uint32_t q = 0; q < parts; ++q)
                            pending.push_back({i, (uint32_t)((uint64_t)N1 * q / parts),
                                               (uint32_t)((uint64_t)N1 * (q + 1) / parts)});
                        parts_left[i] = parts;
                    } else if ((st = hand_over(i, 2)) != VX_OK) {
                        break;
                    }
                }
            for (const Part &pt : taken)
                if (--parts_left[pt.plot] == 0) {
                    const uint32_t i = pt.plot;
                    const uint32_t N1 = 1u << (plan[i].pre[1] + plan[i].D[1]);
                    if ((st = claimed_regions(plan[i], lay[i], buffers[i].workspace, 2, 0, N1, s)) != VX_OK) break;
                    if ((st = hand_over(i, 3)) != VX_OK) break;
                }
        }
    }
    // Join every used lane back into the caller's stream, also on failure, so
    // the caller's stream never runs ahead of work already enqueued.
    for (int l = 0; l < kBatchLanes; ++l) {
        if (!used[l]) continue;
        VX_HIP(hipEventRecord(ln->join[l], ln->s[l]), "batch join");
        VX_HIP(hipStreamWaitEvent(s, ln->join[l], 0), "batch join wait");
    }
    if (st == VX_OK) g_err[0] = 0;
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// vx_plot_noalloc: vx_plot whose workspace is a fixed array the library
// holds on every device it runs on, for callers that cannot allocate.  In
// host code the array's name is no device address: every host use goes
// through the address hipGetSymbolAddress gives for the current device.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[VX_NOALLOC_WORKSPACE_BYTES];

namespace {

struct ScratchSlot {
    bool ready = false;
    void *ptr = nullptr;
};

ScratchSlot g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The current device's copy of `scratch`, looked up once per device.
vx_status scratch_for_current_device(void **out) {
    int dev = 0;
    VX_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(VX_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> guard(g_scratch_mu);
    ScratchSlot &sl = g_scratch[dev];
    if (!sl.ready) {
        void *p = nullptr;
        VX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p || !aligned(p, 256)) return fail(VX_ERR_DEVICE, "the library's workspace array has no usable address");
        sl.ptr = p;
        sl.ready = true;
    }
    *out = sl.ptr;
    return VX_OK;
}

}  // namespace

extern "C" {

vx_status vx_plot_noalloc(const vx_plot_params *params, const vx_plot_buffers *buffers, const vx_tuning *tuning,
                          uint32_t *d_status, void *stream) {
    if (!buffers) return fail(VX_ERR_INVALID_ARG, "buffers is NULL");
    if (buffers->workspace || buffers->workspace_bytes)
        return fail(VX_ERR_INVALID_ARG,
                    "vx_plot_noalloc uses the library's own workspace: buffers->workspace must be NULL and "
                    "workspace_bytes 0");
    if (d_status && !aligned(d_status, 4)) return fail(VX_ERR_INVALID_ARG, "misaligned d_status");
    Plan P;
    vx_status st = make_plan(params, tuning, &P);
    if (st != VX_OK) return st;
    const size_t need = layout(P, VX_CALL_PLOT).total;
    if (need > (size_t)VX_NOALLOC_WORKSPACE_BYTES) {
        char msg[200];
        snprintf(msg, sizeof(msg),
                 "this plot needs %zu workspace bytes; vx_plot_noalloc holds %zu (k <= 22 at the default "
                 "tuning)", need, (size_t)VX_NOALLOC_WORKSPACE_BYTES);
        return fail(VX_ERR_WORKSPACE, msg);
    }
    void *ws = nullptr;
    st = scratch_for_current_device(&ws);
    if (st != VX_OK) return st;
    vx_plot_buffers b = *buffers;
    b.workspace = ws;
    b.workspace_bytes = VX_NOALLOC_WORKSPACE_BYTES;
    // No pipelining: its second stream would be created on first use.
    st = plot_impl(params, &b, tuning, nullptr, stream, false);
    if (st != VX_OK) return st;
    if (d_status)
        VX_HIP(hipMemcpyAsync(d_status, ws, sizeof(uint32_t), hipMemcpyDeviceToDevice, (hipStream_t)stream),
               "status copy");
    g_err[0] = 0;
    return VX_OK;
}

vx_status vx_read_status(const void *d_workspace, uint32_t *h_status, void *stream) {
    if (!d_workspace || !h_status) return fail(VX_ERR_INVALID_ARG, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    VX_HIP(hipMemcpyAsync(h_status, d_workspace, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "status copy");
    VX_HIP(hipStreamSynchronize(s), "status sync");
    g_err[0] = 0;
    return VX_OK;
}

}  // extern "C"
