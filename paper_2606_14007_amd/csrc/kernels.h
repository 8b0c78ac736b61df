// Launchers of the plotter kernels (defined in kernels.hip).  Internal to
// libvx; the public boundary is include/vx.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define VXK_BUCKET_BITS 24
#define VXK_NUM_BUCKETS (1u << VXK_BUCKET_BITS)
#define VXK_DEV_STATUS_GROUP_TOO_LARGE 0x1u
#define VXK_DEV_STATUS_LOOKBACK_TIMEOUT 0x2u
#define VXK_DEV_STATUS_REGION_OVERFLOW 0x4u

namespace vxk {

constexpr int kMaxDigitBits = 11;     // widest partition digit (LDS histograms)
constexpr int kGroupCapMax = 3072;    // records a sort group may hold in LDS
// Default group capacity: the sort kernel for it fits four work-groups
// on a CU (LDS and 64 VGPRs), against three for kGroupCapMax.
constexpr int kGroupCapFast = 2560;
constexpr uint32_t kFallbackMax = 1u << 20;  // largest group the fallback sorts
constexpr int kMatchChunkBitsMax = 11;  // match chunk = 2^bits records (LDS capacity 2048)
// Hash fused with the first partition pass: sub-tiles of 256 * 8 nonces,
// at most 2^8 digits.
constexpr int kHashScatterItems = 8;
constexpr int kHashScatterMaxBits = 8;
constexpr int kHashScatterMaxDigits = 1 << kHashScatterMaxBits;
constexpr uint32_t kHashScatterSub = 256u * kHashScatterItems;
constexpr int kClaimMaxBits = 9;  // widest digit of a claiming scatter

hipError_t launch_reset(uint32_t *words, uint32_t n, hipStream_t s);

// Hash of nonce slices beside the next partition pass of slices hashed in an
// earlier launch (k_hash_pass).  Items are sub-tiles of kHashScatterSub
// records.
struct HashSliceDesc {       // hash nonces [nonce0, nonce0 + n), file them by the first digit
    uint32_t key[8];         // plot key, little-endian words
    uint64_t nonce0, n;
    uint64_t *keys;          // region d of the slice: records [d * R, (d + 1) * R)
    uint32_t *nonces;
    uint32_t *fill;          // records filed per region (zero before the slice's launch)
    uint32_t *status;        // device status word of the plot
    uint32_t bits, R;        // first-digit bits (<= kHashPassMaxBits), region capacity
    uint32_t items;          // ceil(n / kHashScatterSub)
    uint32_t pad;
};
struct PassSliceDesc {       // file the regions of a hashed slice by the next digit
    const uint64_t *keys;    // nin regions of R_in records
    const uint32_t *nonces;
    const uint32_t *fill;    // their fills (clamped to R_in)
    uint64_t *out_keys;      // region r * 2^bits + d of the output: [region * R_out, + R_out)
    uint32_t *out_nonces;
    uint32_t *out_fill;      // shared by every slice of the plot (zero before its first slice)
    uint32_t *status;
    uint32_t R_in, per;      // per: sub-tiles per input region = ceil(R_in / kHashScatterSub)
    uint32_t shift, bits;    // digit = (key >> shift) & (2^bits - 1), bits <= kHashPassMaxBits
    uint32_t R_out;
    uint32_t items;          // nin * per
    uint32_t r0;             // first input region's index in the plot's second-pass regions
    uint32_t pad;
};
constexpr int kHashPassMaxSlices = 8;
struct HashPassList {
    HashSliceDesc h[kHashPassMaxSlices];
    PassSliceDesc p[kHashPassMaxSlices];
    uint32_t nh, np;
    uint32_t h_items, p_items;  // totals over the lists
    uint64_t h_frac;            // ceil(h_items * 2^32 / (h_items + p_items))
    uint32_t sub;               // records per item: kHashScatterSub (0: the same; 256-thread
                                // work-groups) or kHashPassWideSub (512 threads)
    uint32_t pad;
};
constexpr uint32_t kHashPassWideSub = 512u * kHashScatterItems;
constexpr int kHashPassMaxBits = 8;  // widest digit of a sliced hash's two passes
constexpr int kPipeMaxBits = 7;      // widest digit of k_pipe's filing items

// Where a group's records come from: in place (keys == NULL) or records
// [lo[g], hi[g]) of keys / nonces (the last partition pass's regions).
struct GroupIn {
    const uint64_t *keys;
    const uint32_t *nonces;
    const uint32_t *lo;
    const uint32_t *hi;
};

// What one group sort needs besides the group's index (one plot).
struct SortArgs {
    uint64_t *keys;               // Table 1
    uint32_t *nonces;
    GroupIn in;
    const uint32_t *gstart;
    uint32_t *offsets;
    uint32_t *ovf_count, *ovf_list;
    uint8_t *pcnt;                // may be NULL
    unsigned long long *csum;     // may be NULL
    uint64_t T;
    uint32_t G, cap, n_total, cb;
};

// What one match chunk needs besides the chunk's index (one plot).
struct MatchArgs {
    uint32_t key[8];
    const uint64_t *keys;       // Table 1
    const uint32_t *nonces;
    const uint8_t *pcnt;        // pair count of every record (one byte)
    const uint64_t *chunk_base; // Table-2 index of each chunk's first pair
    uint4 *t2;
    uint64_t cap;
    uint64_t T;
    uint32_t n_total, cb;
};

// One launch of a software-pipelined plot or batch (k_pipe): lists of
// hash slices (H), partition-pass slices (P), group ranges to sort (S) and
// record ranges to match (M), whose inputs earlier launches finished.
constexpr int kPipeMaxLists = 4;
constexpr int kPipeBlock = 512;
constexpr uint32_t kPipeSub = 4096;  // records of a filing sub-tile (H and P items)
struct PipeSortDesc {
    SortArgs a;
    uint32_t g0, items;      // groups [g0, g0 + items)
};
struct PipeMatchDesc {
    MatchArgs a;
    const uint32_t *r_lo, *r_hi;  // the chunks owned by records [*r_lo, *r_hi) (to the end when last)
    uint32_t last;
    uint32_t items;               // an upper bound of their number
};
struct PipeList {
    HashSliceDesc h[kPipeMaxLists];
    PassSliceDesc p[kPipeMaxLists];
    PipeSortDesc s[kPipeMaxLists];
    PipeMatchDesc m[kPipeMaxLists];
    uint32_t n[4];       // descriptors of each kind: H, P, S, M
    uint32_t items[4];   // items of each kind
    uint64_t frac[3];    // ceil(items[r] * 2^32 / (items of kinds >= r)), r = 0..2
};
// One launch over the list, which is first stored at d_list (device memory,
// free again once the launch is done); *ticket zero at launch.
hipError_t launch_pipe(const PipeList &L, PipeList *d_list, uint32_t *ticket, hipStream_t s);
// One launch over the list; *ticket zero at launch.
hipError_t launch_hash_pass(const HashPassList &L, uint32_t *ticket, hipStream_t s);
// gstart[d] (d <= nd) over the per-slice regions of a sliced hash.
hipError_t launch_region_scan_slices(const uint32_t *fill, uint32_t slices, uint32_t stride, uint32_t nd,
                                     uint32_t R, uint32_t *gstart, hipStream_t s);
// Chunked plots: hash all n nonces, keep keys whose top pbits bits are
// `prefix`; *count (zero at launch) receives how many (records past cap are
// not written).
hipError_t launch_hash_filter(const uint32_t key_words[8], uint64_t n, uint32_t tiles, uint64_t chunk,
                              uint32_t pbits, uint32_t prefix, uint64_t *keys, uint32_t *nonces, uint64_t cap,
                              unsigned long long *count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
// Stores n <= 16 words (passed by value) at p.
hipError_t launch_put_words(uint32_t *p, const uint32_t *values, uint32_t n, hipStream_t s);
// Plot hash fused with the first partition pass (2^bits digits, bits <=
// kHashScatterMaxBits): record of digit d goes to region d = [d * R,
// (d + 1) * R) of keys / nonces; fill[d] (zero at launch) counts them.
hipError_t launch_hash_scatter(const uint32_t key_words[8], uint64_t n, uint32_t bits, uint32_t R, uint64_t *keys,
                               uint32_t *nonces, uint32_t *fill, uint32_t *status, hipStream_t s);
// Region bounds and output starts of the regions (one work-group).
hipError_t launch_region_scan(const uint32_t *fill, uint32_t nd, uint32_t R, uint32_t *seg_lo, uint32_t *seg_hi,
                              uint32_t *gstart, hipStream_t s);
hipError_t launch_hash_table1(const uint32_t key_words[8], uint64_t n, uint32_t tiles, uint64_t chunk,
                              uint64_t *keys, uint32_t *hist, uint32_t hist_bits, hipStream_t s);
hipError_t launch_hist_chunks(const uint64_t *keys, uint64_t n, uint32_t tiles, uint64_t chunk,
                              uint32_t shift, uint32_t bits, uint32_t *hist, hipStream_t s);
// Segmented launches: segment s covers [seg[s], seg_end[s]); seg_end = NULL
// means back-to-back segments ending at seg[s + 1].
hipError_t launch_hist_segments(const uint64_t *keys, const uint32_t *seg, const uint32_t *seg_end, uint32_t nseg,
                                uint32_t q, uint32_t shift, uint32_t bits, uint32_t *hist, hipStream_t s);
hipError_t launch_colscan(const uint32_t *hist, uint32_t *off, uint32_t nseg, uint32_t rps,
                          uint32_t ncol, const uint32_t *seg_base, uint32_t *gstart, uint32_t n_groups,
                          uint32_t n_total, hipStream_t s);
hipError_t launch_scatter_chunks(const uint64_t *in_keys, const uint32_t *in_nonces,
                                 uint64_t *out_keys, uint32_t *out_nonces, const uint32_t *off,
                                 uint64_t n, uint32_t tiles, uint64_t chunk, uint32_t shift,
                                 uint32_t bits, hipStream_t s);
hipError_t launch_scatter_segments(const uint64_t *in_keys, const uint32_t *in_nonces,
                                   uint64_t *out_keys, uint32_t *out_nonces, const uint32_t *off,
                                   const uint32_t *seg, const uint32_t *seg_end, uint32_t nseg, uint32_t q,
                                   uint32_t shift, uint32_t bits, hipStream_t s);
// Scatter that claims room in fixed regions instead of using a histogram
// scan (bits <= kClaimMaxBits): record of segment s and digit d goes to
// region s * 2^bits + d = [region * R, + R) of out; fill[region] (zero at
// launch) counts them, overflow raises VXK_DEV_STATUS_REGION_OVERFLOW.
hipError_t launch_scatter_claim(const uint64_t *in_keys, const uint32_t *in_nonces, uint64_t *out_keys,
                                uint32_t *out_nonces, const uint32_t *seg, const uint32_t *seg_end, uint32_t nseg,
                                uint32_t q, uint32_t shift, uint32_t bits, uint32_t *fill, uint32_t R,
                                uint32_t *status, hipStream_t s);
// Clamps the counts of regions [r0, r0 + nregions) (fill, seg_lo and seg_hi
// point at region r0) to R in place and writes their bounds.
hipError_t launch_region_bounds(uint32_t *fill, uint32_t r0, uint32_t nregions, uint32_t R, uint32_t *seg_lo,
                                uint32_t *seg_hi, hipStream_t s);
// Group sorts write group g to keys / nonces at gstart[g].  They read it in
// place, or (in_keys != NULL) from records [in_lo[g], in_hi[g]) of in_keys /
// in_nonces.
hipError_t launch_groupsort(uint64_t *keys, uint32_t *nonces, const uint64_t *in_keys, const uint32_t *in_nonces,
                            const uint32_t *in_lo, const uint32_t *in_hi, const uint32_t *gstart, uint32_t G, uint32_t cap,
                            uint32_t *offsets, uint32_t n_total, uint32_t *ovf_count, uint32_t *ovf_list, uint64_t T,
                            uint8_t *pcnt, uint32_t g0, uint32_t gcount, uint32_t *ticket, uint64_t *csum,
                            uint32_t cb, hipStream_t s);
hipError_t launch_group_fallback(uint64_t *keys, uint32_t *nonces, const uint64_t *in_keys,
                                 const uint32_t *in_nonces, const uint32_t *in_lo, const uint32_t *in_hi,
                                 uint64_t *scr_keys,
                                 uint32_t *scr_nonces, const uint32_t *gstart, uint32_t G,
                                 uint32_t *offsets, const uint32_t *ovf_count, const uint32_t *ovf_list,
                                 uint32_t *status, uint64_t T, uint8_t *pcnt, uint64_t *csum, uint32_t cb,
                                 hipStream_t s);
hipError_t launch_match_count(const uint64_t *keys, uint32_t n_total, uint32_t chunk_bits, uint64_t T,
                              uint64_t *counts, uint8_t *pcnt, hipStream_t s);
// Ranged launches: the records [*r_lo, *r_hi) (device words; NULL = all
// records) own the match chunks [*r_lo >> bits, *r_hi >> bits), or up to
// the last chunk when `last`; max_chunks bounds their number (grid size).
hipError_t launch_chunk_sums(const uint8_t *pcnt, const uint64_t *keys, uint32_t n_total, uint32_t chunk_bits,
                             uint64_t T, uint64_t *counts, const uint32_t *r_lo, const uint32_t *r_hi,
                             uint32_t last, uint32_t max_chunks, hipStream_t s);
hipError_t launch_scan_range(const uint64_t *counts, uint64_t *bases, uint32_t n_total, uint32_t chunk_bits,
                             const uint32_t *r_lo, const uint32_t *r_hi, uint32_t last, uint64_t *acc,
                             uint64_t *t2_count, hipStream_t s);
hipError_t launch_zero_u64(uint64_t *p, uint32_t n, hipStream_t s);
// Fused group sort + match + Table-2 hash of all 2^G groups (look-back
// words[2^G] zero at launch, *ticket zero at launch).  Groups are read in
// place or, with in_keys, gathered from records [in_lo[g], in_hi[g]).
hipError_t launch_group_match(const uint32_t key_words[8], uint64_t *keys, uint32_t *nonces, const uint64_t *in_keys,
                              const uint32_t *in_nonces, const uint32_t *in_lo, const uint32_t *in_hi,
                              uint64_t *scr_keys, uint32_t *scr_nonces, const uint32_t *gstart, uint32_t G,
                              uint32_t cap, uint32_t *offsets, uint32_t n_total, uint64_t T, uint32_t *ticket,
                              uint64_t *words, uint32_t *dev_status, void *t2, uint64_t t2cap, uint64_t *t2_count,
                              uint32_t spin_limit, hipStream_t s);
hipError_t launch_scan_u64(const uint64_t *in, uint32_t n, uint64_t *out, uint64_t *part,
                           uint64_t *total, hipStream_t s);
uint32_t scan_parts(uint32_t n);
// wg_per_cu: 0 = as many work-groups as fit on the device, else at most
// that many per CU (to leave room for kernels of another stream).
hipError_t launch_match_emit(const uint32_t key_words[8], const uint64_t *keys, const uint32_t *nonces,
                             const uint8_t *pcnt, uint32_t n_total, uint32_t chunk_bits, uint64_t T,
                             const uint64_t *chunk_base, void *t2, uint64_t cap, const uint32_t *r_lo,
                             const uint32_t *r_hi, uint32_t last, uint32_t max_chunks, uint32_t wg_per_cu,
                             uint32_t *ticket, hipStream_t s);

}  // namespace vxk
