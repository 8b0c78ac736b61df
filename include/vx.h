/*
 * vx.h -- C ABI of the MI355X VaultX plotter hot path (libvx.so).
 *
 * What is computed (VaultxGPU paper, sections I-A, II-B, III-A, III-B):
 *   Table 1: every nonce n in [0, 2^k) is hashed with keyed BLAKE3 under the
 *            256-bit plot key; the first 8 output bytes, read big-endian,
 *            form key64(n).  Records (key64, n) are filed into 2^24 buckets
 *            by the 24-bit prefix key64 >> 40 and each bucket is sorted by
 *            hash value, ties by nonce.
 *   Table 2: inside each bucket, every pair i < j (Table-1 order) with
 *            key64[j] - key64[i] < T is hashed with keyed BLAKE3 over
 *            LE32(nonce_i) || LE32(nonce_j) into a 16-byte record.
 * Readings of what the paper leaves open: nonce = 4-byte little-endian u32;
 * hash kept = 8 bytes, big-endian u64; default T = 2^(64-k), the expected
 * gap between neighbouring keys; strict "<"; pairs never cross buckets;
 * Table 2 in order of i, then j.
 *
 * Conventions for every call:
 *  - Pointers named d_* are DEVICE pointers owned by the caller; the library
 *    never frees them and keeps none after the enqueued work completes.
 *    Host pointers (params, buffers, tuning structs) are read during the
 *    call only.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call only
 *    enqueues work on it and returns; outputs are valid once the stream has
 *    reached that point.
 *  - Argument and size errors are returned synchronously and enqueue
 *    nothing.  A failed HIP launch returns VX_ERR_DEVICE.  vx_last_error()
 *    gives a message for the calling thread's last failure.
 *  - Data-dependent conditions are reported on the device: Table-2 overflow
 *    as *d_t2_count > t2_capacity (records past the capacity are not
 *    written), and degenerate inputs the sort cannot place (see
 *    vx_read_status) in a status word at the start of the workspace.
 *  - Outputs are deterministic and bit-exact: they do not depend on tuning,
 *    on the stream, or on other work running at the same time.
 *  - Sizes: k in [1, 31]; 2^k records; offsets have 2^24 + 1 entries.
 */
#ifndef VX_H
#define VX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VX_OK = 0,
    VX_ERR_INVALID_ARG = 1,   /* bad k, bucket_bits, null or misaligned pointer */
    VX_ERR_WORKSPACE = 2,     /* workspace smaller than vx_workspace_bytes() */
    VX_ERR_DEVICE = 3,        /* a HIP call failed; see vx_last_error() */
    VX_ERR_OUT_OF_MEMORY = 4, /* reserved for callers that allocate through the library */
    VX_ERR_UNSUPPORTED = 5,   /* a tuning value outside its supported range */
    VX_ERR_IO = 6,            /* writing a plot file failed (vx_egress_*) */
} vx_status;

/* Device status word bits (vx_read_status). */
#define VX_DEV_STATUS_GROUP_TOO_LARGE 0x1u /* a sort group exceeded the fallback limit */
#define VX_DEV_STATUS_LOOKBACK_TIMEOUT 0x2u /* vx_plot: a Table-2 base wait hit its bound */
#define VX_DEV_STATUS_REGION_OVERFLOW 0x4u /* vx_plot, staged plots: a partition region
                                              overflowed (about 8 standard deviations above its
                                              expected fill; Table 1 is then incomplete) */

#define VX_BUCKET_BITS 24
#define VX_NUM_BUCKETS (1u << VX_BUCKET_BITS)

/* One plot.  key: the 256-bit plot key (paper sec. III-B), used as eight
 * little-endian words.  k: log2 of the number of nonces.  bucket_bits: must
 * be 24 (2^24 buckets, paper sec. I-A).  match_threshold: T of the match
 * predicate; vx_default_threshold(k) gives the paper-scale default. */
typedef struct {
    uint8_t key[32];
    uint32_t k;
    uint32_t bucket_bits;
    uint64_t match_threshold;
} vx_plot_params;

/* One Table-2 record, 16 bytes, little-endian fields. */
typedef struct {
    uint32_t nonce_a; /* nonce of the earlier record in Table-1 order */
    uint32_t nonce_b; /* nonce of the later record */
    uint64_t hash2;   /* BE64 of the first 8 bytes of keyed BLAKE3(LE32 a || LE32 b) */
} vx_t2_record;

/* Buffers of a whole plot (vx_plot).  All device pointers, caller-owned:
 *  t1_keys[2^k] (u64, 8-byte aligned), t1_nonces[2^k] (u32),
 *  bucket_offsets[2^24 + 1] (u32; offsets[b] = index of the first Table-1
 *  record of bucket b, offsets[2^24] = 2^k),
 *  t2[t2_capacity] records (16-byte aligned), t2_count: one device u64 that
 *  receives |Table 2| (which may exceed t2_capacity),
 *  workspace: at least vx_workspace_bytes(params, VX_CALL_PLOT, tuning)
 *  bytes, 256-byte aligned. */
typedef struct {
    uint64_t *t1_keys;
    uint32_t *t1_nonces;
    uint32_t *bucket_offsets;
    vx_t2_record *t2;
    uint64_t t2_capacity;
    uint64_t *t2_count;
    void *workspace;
    size_t workspace_bytes;
} vx_plot_buffers;

/* Implementation parameters.  None of them changes any output (except
 * region_pct below 100, a test hook); they only move work between kernels.  Zero in any field selects the built-in
 * default for the plot's k.  The group_bits leading key bits are split over
 * at most three partition passes of at most 11 bits each. */
typedef struct {
    uint32_t group_bits;   /* sort groups = 2^group_bits key prefixes, 1..24 */
    uint32_t pass1_bits;   /* digit bits of the first partition pass, 1..11 */
    uint32_t group_cap;    /* records a group may hold in LDS, 64..3072 (0: 2560, or 3072 with fused_sort_match) */
    uint32_t h1_tiles;     /* work-groups of a separate hash and first partition pass (a plot whose
                              hash does the first pass sizes that kernel's grid itself) */
    uint32_t match_chunk_bits; /* match works on chunks of 2^bits Table-1 records, 6..11 */
    uint32_t pass2_bits;   /* digit bits of the second pass (a third takes the rest) */
    uint32_t fused_sort_match; /* plot: nonzero runs sort, match and Table-2 hash as one kernel */
    uint32_t pipeline_slices;  /* vx_plot: 0 or 1 = no pipelining (default); 2..16 = slices of the
                                  work after the first partition pass, whose matches run on a
                                  second (internal) stream while later slices are partitioned and
                                  sorted */
    uint32_t separate_hash;    /* plot: nonzero keeps the hash and the first partition pass as two
                                  kernels (by default a plot with two or more passes hashes and
                                  files records by their first digit in one kernel) */
    uint32_t region_pct;       /* plot, staged plots: capacity of the partition regions in percent of
                                  the default (0 = 100).  The one exception to "no output
                                  changes": below 100 regions can overflow, which sets
                                  VX_DEV_STATUS_REGION_OVERFLOW (for tests of that report) */
    uint32_t hash_slices;      /* vx_plot: 1 = hash the plot in one launch; 2..32 = hash it in that
                                  many nonce slices, each launch filing the previous slice's records
                                  by the second digit beside the next slice's hash (plots whose two
                                  leading digits fit 7 bits each); 0 = the default for k */
    uint32_t tail_slices;      /* vx_plot: 1 = the third partition pass, the sort and the match as
                                  separate kernels; 2..16 = pipelined over that many slices of the
                                  first pass's segments, one persistent launch per step running the
                                  third pass of one slice, the sort of the previous and the match of
                                  the one before (plots with region passes, group_cap <= 2560 and
                                  digits of at most 7 bits after the second); 0 = the default for k */
    uint32_t batch_shared_hash; /* vx_plot_batch: nonzero lets this plot's hash launches (and its
                                  second and third partition passes) be shared with other plots of
                                  the batch that ask for it -- one persistent launch per step over a
                                  device work list of slices of several plots; 0 (default) runs the
                                  plot on its own, on one of the batch's lanes */
    uint32_t front_passes;     /* vx_plot: partition passes that the launches of a sliced hash file
                                  when the plot has three: 2 = the first two (the third runs as a
                                  separate scatter); 3 = all three, launch i also filing slice i - 2
                                  by the third digit (a third digit of at most 7 bits, and neither
                                  tail_slices nor batch_shared_hash); 0 = 3 where the plan allows */
    uint32_t front_subtile;    /* vx_plot: records per work item of a sliced hash's launches, 2048
                                  (256-thread work-groups) or 4096 (512 threads: each digit's run
                                  twice as long); 0 = 4096 where the launches file three
                                  passes, else 2048 */
} vx_tuning;

enum { VX_CALL_BUCKET_SORT = 1, VX_CALL_MATCH = 2, VX_CALL_PLOT = 3 };

/* 2^(64-k): the expected gap between neighbouring keys of a k-plot. */
uint64_t vx_default_threshold(uint32_t k);

/* Workspace bytes a call needs for these params and tuning (tuning may be
 * NULL).  Returns 0 for invalid params. */
size_t vx_workspace_bytes(const vx_plot_params *params, int which_call, const vx_tuning *tuning);

/* Number of MSD partition passes (1..3) that the plan for these params and
 * tuning (may be NULL) makes over Table 1 before sorting inside groups --
 * what a caller needs to account the bytes a sort moves.  No device work.
 * Returns 0 for invalid params or tuning. */
uint32_t vx_partition_passes(const vx_plot_params *params, const vx_tuning *tuning);

/* Nonce slices in which vx_plot hashes a plot with these params and tuning
 * (may be NULL): 1 = one launch; s >= 2 = s launches, each filing the
 * previous slice's records by the second digit beside its own hash, so the
 * first two partition passes are done by then.  No device work.  Returns 0
 * for invalid params or tuning. */
uint32_t vx_hash_slices(const vx_plot_params *params, const vx_tuning *tuning);

/* Partition passes that vx_plot's hash launches file for these params and
 * tuning (may be NULL): 0 = none (a separate hash kernel), 1 = the first, 2
 * or 3 = that many, in nonce slices (vx_hash_slices >= 2).  No device work.
 * Returns 0 also for invalid params or tuning. */
uint32_t vx_front_passes(const vx_plot_params *params, const vx_tuning *tuning);

/* Slices over which vx_plot pipelines the work after the first two
 * partition passes (the third pass, the sort and the match, in one
 * persistent launch per step): 1 = not pipelined.  No device work.  Returns
 * 0 for invalid params or tuning. */
uint32_t vx_tail_slices(const vx_plot_params *params, const vx_tuning *tuning);

/* A Table-2 capacity that holds |Table 2| of a k-plot with threshold T with
 * overwhelming probability (expectation plus a generous margin). */
uint64_t vx_t2_capacity_hint(uint32_t k, uint64_t threshold);

/* Table-1 hashing (paper sec. III-A, III-B: one hash per nonce, all 2^k
 * nonces): d_keys[n] = key64(n) for n in [0, 2^k), in nonce order. */
vx_status vx_hash_table1(const vx_plot_params *params, uint64_t *d_keys, void *stream);

/* Bucketing and in-bucket sort (paper sec. III-A, III-B; sort by hash value
 * inside each of the 2^24 buckets): from nonce-order hashes d_keys[2^k]
 * (record n has nonce n) to Table 1 sorted by (key64, nonce) in
 * d_t1_keys / d_t1_nonces, and d_offsets[2^24 + 1].  d_keys is read only and
 * must not overlap the outputs. */
vx_status vx_bucket_sort(const vx_plot_params *params, const uint64_t *d_keys,
                         uint64_t *d_t1_keys, uint32_t *d_t1_nonces, uint32_t *d_offsets,
                         void *d_workspace, size_t workspace_bytes, const vx_tuning *tuning,
                         void *stream);

/* Match and Table-2 hashing (paper sec. II-B, III-A: pairs within the
 * threshold, hashed into Table-2 records) over a sorted Table 1.  Writes
 * min(|T2|, t2_capacity) records in canonical order and |T2| to
 * *d_t2_count.  d_offsets must be the table's bucket offsets (it is checked
 * for NULL; bucket boundaries are read from the keys themselves). */
vx_status vx_match_table2(const vx_plot_params *params, const uint64_t *d_t1_keys,
                          const uint32_t *d_t1_nonces, const uint32_t *d_offsets,
                          vx_t2_record *d_t2, uint64_t t2_capacity, uint64_t *d_t2_count,
                          void *d_workspace, size_t workspace_bytes, const vx_tuning *tuning,
                          void *stream);

/* Whole plot (paper sec. III-A pipeline without the host copy and disk
 * write): the same outputs as vx_match_table2(vx_bucket_sort(
 * vx_hash_table1())). */
vx_status vx_plot(const vx_plot_params *params, const vx_plot_buffers *buffers,
                  const vx_tuning *tuning, void *stream);

/* Number of events vx_plot_with_events records. */
#define VX_PLOT_EVENTS 7

/* vx_plot that also records caller-created hipEvent_t handles on `stream`
 * at its stage boundaries, for per-stage timing: events[0] before the hash
 * kernel (after the small workspace-header reset); events[1] after the Table-1 hash; [2] after partition pass 1;
 * [3] after partition pass 2 (no kernels between [2] and [3] when the plot
 * needs one pass); [4] after the in-group sort; [5] after the match count
 * and its scan; [6] after the match and Table-2 hash.  Outputs and errors
 * are those of vx_plot; events must not be NULL. */
vx_status vx_plot_with_events(const vx_plot_params *params, const vx_plot_buffers *buffers,
                              const vx_tuning *tuning, void *const *events, void *stream);

/* n independent plots (params[i], buffers[i]) as one unit of work on
 * `stream`: the call forks the stream into a few internal lane streams, runs
 * each lane's plots in order, and joins the lanes back into `stream`, so
 * that kernels of different plots overlap on the device and a caller can
 * capture the whole batch into one HIP graph.  Plots whose buffers share the
 * same workspace run one after another in list order (so one workspace per
 * lane suffices); other buffers must not overlap.  Each output equals
 * vx_plot(params[i], buffers[i]).  tuning is NULL (built-in defaults per k)
 * or an array of n entries.  All plots (parameters, buffers, workspaces) are
 * validated before anything is enqueued.  The status word of each workspace
 * (vx_read_status) is cleared once per batch and then collects the device
 * status bits of every plot that used it.  The lane streams are shared per
 * device: batches on one device must not be captured from two threads at
 * once. */
vx_status vx_plot_batch(const vx_plot_params *params, const vx_plot_buffers *buffers,
                        uint32_t n, const vx_tuning *tuning, void *stream);

/* Bytes of the workspace array that libvx holds on each device for
 * vx_plot_noalloc (enough for k <= 22 at the default tuning). */
#define VX_NOALLOC_WORKSPACE_BYTES (128u << 20)

/* vx_plot for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace is a fixed array of VX_NOALLOC_WORKSPACE_BYTES that the library
 * holds on each device it runs on, from the first call on that device until
 * the process ends; the call itself allocates nothing.  buffers->workspace
 * must be NULL and workspace_bytes 0; the other buffers are the caller's, as
 * for vx_plot, and the outputs equal vx_plot's.  A plot whose workspace
 * (vx_workspace_bytes) exceeds the array returns VX_ERR_WORKSPACE and
 * enqueues nothing.  d_status: NULL, or one caller-owned device u32 that
 * receives the plot's device status word (VX_DEV_STATUS_*) at its end.
 * Every call on one device shares that device's array: calls that can
 * overlap on one device (other streams, other host threads) race and must
 * be serialised by the caller. */
vx_status vx_plot_noalloc(const vx_plot_params *params, const vx_plot_buffers *buffers,
                          const vx_tuning *tuning, uint32_t *d_status, void *stream);

/* ------------------------------------------------------------------------
 * Chunked plots.  A plot can be made in 2^chunk_bits chunks of its bucket
 * space: chunk r holds the buckets whose top chunk_bits bits equal r
 * (buckets [r * 2^(24 - chunk_bits), (r + 1) * 2^(24 - chunk_bits))).  Each
 * chunk hashes every nonce of the plot, keeps its own records, and sorts and
 * matches them like a whole plot; pairs never cross buckets (sec. III-A),
 * so Table 2 of a chunk is exactly that of its buckets.  The whole plot's
 * Table 1 and Table 2 are the chunks' in chunk order, and its bucket offsets
 * those of each chunk plus the records of the chunks before it.  Device
 * memory is then bounded by one chunk, and k = 32 -- 2^32 records, more
 * than the 32-bit offsets of a whole plot hold -- is made in two or more
 * chunks (the paper plots up to K=31 and names larger plots as future work,
 * sec. V).  k may be 32 in these calls; nonces stay 4-byte little-endian. */

/* Table-1 records a chunk holds with overwhelming probability (expectation
 * plus 8 standard deviations plus 4096), or 0 if that reaches 2^32 or the
 * arguments are out of range (k in [1, 32], chunk_bits in [0, 8] and at most
 * k).  *t2_capacity (may be NULL) receives the matching Table-2 capacity for
 * threshold T. */
uint64_t vx_chunk_capacity_hint(uint32_t k, uint32_t chunk_bits, uint64_t threshold, uint64_t *t2_capacity);

/* Workspace bytes of vx_plot_chunk for up to t1_capacity records (0 for
 * invalid arguments or a fused tuning). */
size_t vx_chunk_workspace_bytes(const vx_plot_params *params, uint32_t chunk_bits, uint64_t t1_capacity,
                                const vx_tuning *tuning);

/* Chunk `chunk` of a plot cut by chunk_bits: writes the chunk's Table 1
 * (m records; t1_keys / t1_nonces must hold t1_capacity), its bucket offsets
 * (2^24 + 1 entries; buckets before the chunk's range get 0, those after it
 * m), its Table 2 and count as vx_plot does, and m to *d_t1_count.  Unlike
 * the other calls it synchronises `stream` once, after the hash, to plan
 * the sort for m records.  Returns VX_ERR_WORKSPACE if m exceeds t1_capacity
 * (nothing further is written).  The fused sort + match tuning is not
 * supported here. */
vx_status vx_plot_chunk(const vx_plot_params *params, uint32_t chunk_bits, uint32_t chunk,
                        const vx_plot_buffers *buffers, uint64_t t1_capacity, uint64_t *d_t1_count,
                        const vx_tuning *tuning, void *stream);

/* Staged chunks.  vx_stage_plot hashes every nonce of a plot once and files
 * the records by their first partition digit into a caller-owned device
 * buffer (the stage); vx_plot_staged_chunk then makes chunk r of the plot
 * from the stage, exactly as vx_plot_chunk does (same outputs, same chunk
 * definition), without hashing again.  The stage holds 12 bytes per record
 * plus slack (51.6 GB at k=32), so making 2^chunk_bits chunks costs one hash
 * of the plot instead of 2^chunk_bits.  The stage stays valid until it is
 * overwritten; chunks may be made in any order and more than once.  A stage
 * is made for one key, k, chunk_bits and tuning, and the chunk calls check
 * this.  Overflow of a stage region (fewer than one plot in 10^13) sets
 * VX_DEV_STATUS_REGION_OVERFLOW in the stage's status word (vx_read_status
 * on the stage).  k may be 32; chunk_bits must not exceed the first digit's
 * width (6 bits with three passes, the default from k=29 up). */

/* Bytes of the stage for these parameters, or 0 if they do not allow a
 * staged plot (fused sort + match, separate_hash, or digits out of range). */
size_t vx_stage_bytes(const vx_plot_params *params, uint32_t chunk_bits, const vx_tuning *tuning);

/* Enqueues the stage hash on `stream` (no synchronisation).  d_stage: at
 * least vx_stage_bytes bytes, 256-byte aligned. */
vx_status vx_stage_plot(const vx_plot_params *params, uint32_t chunk_bits, const vx_tuning *tuning, void *d_stage,
                        size_t stage_bytes, void *stream);

/* Workspace bytes of vx_plot_staged_chunk for up to t1_capacity records (use
 * vx_chunk_capacity_hint), or 0. */
size_t vx_staged_chunk_workspace_bytes(const vx_plot_params *params, uint32_t chunk_bits, uint64_t t1_capacity,
                                       const vx_tuning *tuning);

/* Chunk `chunk` of the staged plot: outputs as vx_plot_chunk (Table 1, the
 * offsets relative to the chunk, Table 2 and its count, m in *d_t1_count).
 * Synchronises `stream` once (the record count plans the sort, and the
 * stage's identity is checked: VX_ERR_INVALID_ARG if it was made for other
 * parameters).  VX_ERR_WORKSPACE if m exceeds t1_capacity. */
vx_status vx_plot_staged_chunk(const vx_plot_params *params, uint32_t chunk_bits, uint32_t chunk,
                               const void *d_stage, size_t stage_bytes, const vx_plot_buffers *buffers,
                               uint64_t t1_capacity, uint64_t *d_t1_count, const vx_tuning *tuning, void *stream);

/* Copies the device status word at the start of a workspace used by
 * vx_bucket_sort or vx_plot to *h_status (synchronising `stream`). */
vx_status vx_read_status(const void *d_workspace, uint32_t *h_status, void *stream);

/* Message for the calling thread's last failed call ("" if none). */
const char *vx_last_error(void);

/* ------------------------------------------------------------------------
 * Table-2 egress.  The paper's plotter copies Table 2 to the host and writes
 * it to storage after the kernels (sec. III-A); at K=27..31 that copy and
 * write take most of a plot's time (sec. IV), and overlapping them with the
 * computation is the first item of its future work (sec. V).  A vx_egress
 * streams finished Tables 2 off the device while the caller's stream goes on
 * computing: it owns pinned host staging buffers (`slots` of `slot_bytes`),
 * an internal copy stream and one writer thread, all on the device current
 * at creation.  Each submitted plot becomes one flat plot file appended to
 * the file descriptor, little-endian:
 *   bytes   0..7    magic "VXPLOT01"
 *   bytes   8..11   header bytes (128)      12..15  record bytes (16)
 *   bytes  16..19   k                       20..23  bucket bits (24)
 *   bytes  24..31   match threshold T
 *   bytes  32..39   |Table 2| as counted on the device
 *   bytes  40..47   records that follow: min(|Table 2|, t2_capacity)
 *   bytes  48..79   the 32-byte plot key
 *   bytes  80..83   chunk_bits              84..87  chunk
 *                   (0, 0 for a whole plot; for chunk r of a chunked plot
 *                   the records are the plot's Table 2 restricted to the
 *                   chunk's buckets, and the chunks' files in chunk order
 *                   concatenate to the plot's Table 2)
 *   bytes  88..127  zero
 *   then the records in canonical order, 16 bytes each (vx_t2_record).
 * The egress is not for HIP graph capture. */
typedef struct vx_egress vx_egress;

/* Creates an egress writing to `fd` (an open file descriptor that the caller
 * keeps and closes; -1 discards the bytes, to measure the copy path alone).
 * slot_bytes: a multiple of 16 in [1 MiB, 1 GiB]; slots: 2..64.  Argument
 * errors return before any allocation. */
vx_status vx_egress_create(int fd, size_t slot_bytes, uint32_t slots, vx_egress **out);

/* Queues one plot file.  Once the work enqueued so far on `stream` is done,
 * the writer thread reads *d_t2_count, copies min(*d_t2_count, t2_capacity)
 * records of d_t2 piece by piece on the egress's stream -- overlapping
 * whatever the caller enqueues next -- and appends the header and records to
 * the file.  d_t2 and d_t2_count must not change until vx_egress_wait() has
 * returned for this job.  *job receives its number (1, 2, ... in submission
 * order).  Returns at once. */
vx_status vx_egress_submit(vx_egress *e, const vx_plot_params *params, const vx_t2_record *d_t2,
                           uint64_t t2_capacity, const uint64_t *d_t2_count, void *stream,
                           uint64_t *job);

/* As vx_egress_submit, for the Table 2 of chunk `chunk` of a plot cut by
 * chunk_bits (vx_plot_chunk, vx_plot_staged_chunk): the file header records
 * chunk_bits and chunk.  chunk_bits <= 8 and chunk < 2^chunk_bits. */
vx_status vx_egress_submit_chunk(vx_egress *e, const vx_plot_params *params, uint32_t chunk_bits, uint32_t chunk,
                                 const vx_t2_record *d_t2, uint64_t t2_capacity, const uint64_t *d_t2_count,
                                 void *stream, uint64_t *job);

/* Blocks until jobs 1..job are written (job = 0: all submitted so far).
 * Returns the first error that any job hit (VX_ERR_IO, VX_ERR_DEVICE). */
vx_status vx_egress_wait(vx_egress *e, uint64_t job);

/* Bytes of plot files written (or discarded) so far. */
uint64_t vx_egress_bytes(const vx_egress *e);

/* Waits for every job, stops the writer thread and frees the egress (NULL is
 * a no-op).  Returns the first error any job hit. */
vx_status vx_egress_destroy(vx_egress *e);

#ifdef __cplusplus
}
#endif

#endif /* VX_H */
