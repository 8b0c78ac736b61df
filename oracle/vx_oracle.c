/*
 * VaultX plotter oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the plotter's
 * hot path computes.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library; the product path never does.  It
 * shares no source with the HIP path (no headers, tables or helpers).
 *
 * Sources it is written from:
 *  - The BLAKE3 specification (O'Connor, Aumasson, Neves, Wilcox-O'Hearn,
 *    "BLAKE3: one function, fast everywhere", 2020): compression function
 *    (spec sec. 2.2), modes and flags (2.3), chunk chaining (2.4), the
 *    binary tree of chunks (2.5) and the extendable output (2.6).
 *  - The VaultxGPU paper: Table-1 generation hashes every nonce with keyed
 *    BLAKE3 and files it into one of 2^24 buckets by hash prefix (sec. I-A,
 *    II-B, III-A, III-B); the sort stage orders each bucket by hash value,
 *    and the match stage pairs entries whose distance is below a threshold
 *    to form Table 2 (sec. II-B, III-A).
 *
 * Readings of what the paper leaves open (all fixed here and in the HIP
 * path by the same reading, not by shared code):
 *  - nonce: 4 bytes, little-endian u32 (sec. III-B names a little-endian
 *    nonce; no width is given);
 *  - hash kept per record: the first 8 output bytes, read big-endian into a
 *    u64 "key64" so that numeric order is byte order (the 64-bit sort key
 *    of sec. III-B);
 *  - bucket = key64 >> 40, the 24-bit prefix (2^24 buckets, sec. I-A);
 *  - Table 1 order: by (key64, nonce) ascending; no capacity, no drops;
 *  - match: pairs i < j in Table-1 order inside one bucket with
 *    key64[j] - key64[i] < T (strict, unsigned); default T = 2^(64-k), the
 *    expected gap between neighbouring keys;
 *  - Table 2 record: {nonce_i u32, nonce_j u32, h2 u64} with h2 = the first
 *    8 bytes, big-endian, of keyed BLAKE3 over LE32(nonce_i) || LE32(nonce_j);
 *    records in order of i, then j.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <time.h>

/* ---------------------------------------------------------------------- */
/* BLAKE3, written from the specification.                                 */
/* ---------------------------------------------------------------------- */

/* Spec sec. 2.2: the IV is the SHA-256 initial hash value. */
static const uint32_t B3_IV[8] = {
    0x6A09E667u, 0xBB67AE85u, 0x3C6EF372u, 0xA54FF53Au,
    0x510E527Fu, 0x9B05688Cu, 0x1F83D9ABu, 0x5BE0CD19u,
};

/* Spec sec. 2.2: message word permutation applied between rounds. */
static const int B3_PERM[16] = {2, 6, 3, 10, 7, 0, 4, 13, 1, 11, 12, 5, 9, 14, 15, 8};

/* Spec sec. 2.3, table of flags. */
enum {
    B3_CHUNK_START = 1u << 0,
    B3_CHUNK_END = 1u << 1,
    B3_PARENT = 1u << 2,
    B3_ROOT = 1u << 3,
    B3_KEYED_HASH = 1u << 4,
    B3_DERIVE_KEY_CONTEXT = 1u << 5,
    B3_DERIVE_KEY_MATERIAL = 1u << 6,
};

#define B3_BLOCK_LEN 64
#define B3_CHUNK_LEN 1024

static uint32_t rotr32(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

static uint32_t load_le32(const uint8_t *p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
           ((uint32_t)p[3] << 24);
}

static void store_le32(uint8_t *p, uint32_t x) {
    p[0] = (uint8_t)x;
    p[1] = (uint8_t)(x >> 8);
    p[2] = (uint8_t)(x >> 16);
    p[3] = (uint8_t)(x >> 24);
}

/* Spec sec. 2.2: the quarter-round G mixing four state words and two
 * message words, rotations 16, 12, 8, 7. */
static void b3_g(uint32_t v[16], int a, int b, int c, int d, uint32_t mx, uint32_t my) {
    v[a] = v[a] + v[b] + mx;
    v[d] = rotr32(v[d] ^ v[a], 16);
    v[c] = v[c] + v[d];
    v[b] = rotr32(v[b] ^ v[c], 12);
    v[a] = v[a] + v[b] + my;
    v[d] = rotr32(v[d] ^ v[a], 8);
    v[c] = v[c] + v[d];
    v[b] = rotr32(v[b] ^ v[c], 7);
}

/* Spec sec. 2.2: one round = G on the four columns, then on the four
 * diagonals, message words taken in order m[0..15]. */
void or_b3_round(uint32_t v[16], const uint32_t m[16]) {
    b3_g(v, 0, 4, 8, 12, m[0], m[1]);
    b3_g(v, 1, 5, 9, 13, m[2], m[3]);
    b3_g(v, 2, 6, 10, 14, m[4], m[5]);
    b3_g(v, 3, 7, 11, 15, m[6], m[7]);
    b3_g(v, 0, 5, 10, 15, m[8], m[9]);
    b3_g(v, 1, 6, 11, 12, m[10], m[11]);
    b3_g(v, 2, 7, 8, 13, m[12], m[13]);
    b3_g(v, 3, 4, 9, 14, m[14], m[15]);
}

void or_b3_iv(uint32_t out[8]) { memcpy(out, B3_IV, sizeof(B3_IV)); }

/* Spec sec. 2.2: the compression function.  Returns all 16 output words:
 * out[i] = v[i] ^ v[i+8] and out[i+8] = v[i+8] ^ cv[i]. */
void or_b3_compress(const uint32_t cv[8], const uint8_t block[64], uint64_t counter,
                    uint32_t block_len, uint32_t flags, uint32_t out[16]) {
    uint32_t m[16], v[16], t[16];
    for (int i = 0; i < 16; i++) m[i] = load_le32(block + 4 * i);
    for (int i = 0; i < 8; i++) v[i] = cv[i];
    v[8] = B3_IV[0];
    v[9] = B3_IV[1];
    v[10] = B3_IV[2];
    v[11] = B3_IV[3];
    v[12] = (uint32_t)counter;
    v[13] = (uint32_t)(counter >> 32);
    v[14] = block_len;
    v[15] = flags;
    for (int r = 0; r < 7; r++) {
        or_b3_round(v, m);
        for (int i = 0; i < 16; i++) t[i] = m[B3_PERM[i]];
        memcpy(m, t, sizeof(m));
    }
    for (int i = 0; i < 8; i++) {
        out[i] = v[i] ^ v[i + 8];
        out[i + 8] = v[i + 8] ^ cv[i];
    }
}

/* A node whose final compression has not been done yet (spec sec. 2.5: the
 * root node's last compression is the one that takes the ROOT flag and is
 * repeated with increasing counters for extended output). */
typedef struct {
    uint32_t cv[8];
    uint8_t block[64];
    uint64_t counter;
    uint32_t block_len;
    uint32_t flags;
} b3_node;

static void b3_node_cv(const b3_node *n, uint32_t cv[8]) {
    uint32_t out[16];
    or_b3_compress(n->cv, n->block, n->counter, n->block_len, n->flags, out);
    memcpy(cv, out, 8 * sizeof(uint32_t));
}

/* Spec sec. 2.4: a chunk of at most 1024 bytes is compressed block by block
 * starting from the key words, with the chunk index as counter; the first
 * block carries CHUNK_START and the last CHUNK_END.  An empty input is one
 * empty block. */
static b3_node b3_chunk(const uint32_t key[8], const uint8_t *p, size_t len,
                        uint64_t chunk_index, uint32_t mode) {
    b3_node n;
    memcpy(n.cv, key, sizeof(n.cv));
    size_t nblocks = len == 0 ? 1 : (len + B3_BLOCK_LEN - 1) / B3_BLOCK_LEN;
    for (size_t b = 0; b + 1 < nblocks; b++) {
        uint32_t out[16];
        uint32_t fl = mode | (b == 0 ? B3_CHUNK_START : 0);
        or_b3_compress(n.cv, p + b * B3_BLOCK_LEN, chunk_index, B3_BLOCK_LEN, fl, out);
        memcpy(n.cv, out, sizeof(n.cv));
    }
    size_t off = (nblocks - 1) * B3_BLOCK_LEN;
    memset(n.block, 0, sizeof(n.block));
    memcpy(n.block, p + off, len - off);
    n.block_len = (uint32_t)(len - off);
    n.counter = chunk_index;
    n.flags = mode | (nblocks == 1 ? B3_CHUNK_START : 0) | B3_CHUNK_END;
    return n;
}

/* Spec sec. 2.5: a parent node compresses the two child chaining values as
 * one 64-byte block, counter 0, with the PARENT flag, starting from the
 * key words. */
static b3_node b3_parent(const uint32_t key[8], const uint32_t l[8], const uint32_t r[8],
                         uint32_t mode) {
    b3_node n;
    memcpy(n.cv, key, sizeof(n.cv));
    for (int i = 0; i < 8; i++) {
        store_le32(n.block + 4 * i, l[i]);
        store_le32(n.block + 32 + 4 * i, r[i]);
    }
    n.counter = 0;
    n.block_len = B3_BLOCK_LEN;
    n.flags = mode | B3_PARENT;
    return n;
}

/* Spec sec. 2.5: the left subtree holds the largest power-of-two number of
 * chunks that leaves the right subtree non-empty. */
static b3_node b3_subtree(const uint32_t key[8], const uint8_t *p, size_t len,
                          uint64_t chunk_index, uint32_t mode) {
    if (len <= B3_CHUNK_LEN) return b3_chunk(key, p, len, chunk_index, mode);
    size_t nchunks = (len + B3_CHUNK_LEN - 1) / B3_CHUNK_LEN;
    size_t left_chunks = 1;
    while (left_chunks * 2 < nchunks) left_chunks *= 2;
    size_t left_len = left_chunks * B3_CHUNK_LEN;
    b3_node l = b3_subtree(key, p, left_len, chunk_index, mode);
    b3_node r = b3_subtree(key, p + left_len, len - left_len, chunk_index + left_chunks, mode);
    uint32_t lcv[8], rcv[8];
    b3_node_cv(&l, lcv);
    b3_node_cv(&r, rcv);
    return b3_parent(key, lcv, rcv, mode);
}

/* Spec sec. 2.6: output block t of the root = the root compression with
 * counter t and the ROOT flag, all 16 words little-endian. */
static void b3_root_output(const b3_node *root, uint8_t *out, size_t out_len) {
    uint64_t t = 0;
    while (out_len > 0) {
        uint32_t w[16];
        uint8_t buf[64];
        or_b3_compress(root->cv, root->block, t, root->block_len, root->flags | B3_ROOT, w);
        for (int i = 0; i < 16; i++) store_le32(buf + 4 * i, w[i]);
        size_t take = out_len < 64 ? out_len : 64;
        memcpy(out, buf, take);
        out += take;
        out_len -= take;
        t++;
    }
}

/* Spec sec. 2.3: hash mode uses the IV as key words; keyed_hash mode uses
 * the 32-byte key (eight little-endian words) and sets KEYED_HASH on every
 * compression.  key == NULL selects hash mode. */
void or_b3_hash(const uint8_t *key, const uint8_t *msg, size_t len, uint8_t *out,
                size_t out_len) {
    uint32_t kw[8];
    uint32_t mode = 0;
    if (key) {
        for (int i = 0; i < 8; i++) kw[i] = load_le32(key + 4 * i);
        mode = B3_KEYED_HASH;
    } else {
        memcpy(kw, B3_IV, sizeof(kw));
    }
    b3_node root = b3_subtree(kw, msg, len, 0, mode);
    b3_root_output(&root, out, out_len);
}

/* Spec sec. 2.3: derive_key mode hashes the context string with
 * DERIVE_KEY_CONTEXT from the IV; its 32-byte output becomes the key words
 * for hashing the key material with DERIVE_KEY_MATERIAL. */
void or_b3_derive_key(const char *context, size_t context_len, const uint8_t *material,
                      size_t len, uint8_t *out, size_t out_len) {
    uint32_t kw[8];
    uint8_t ctx_key[32];
    memcpy(kw, B3_IV, sizeof(kw));
    b3_node c = b3_subtree(kw, (const uint8_t *)context, context_len, 0, B3_DERIVE_KEY_CONTEXT);
    b3_root_output(&c, ctx_key, 32);
    for (int i = 0; i < 8; i++) kw[i] = load_le32(ctx_key + 4 * i);
    b3_node root = b3_subtree(kw, material, len, 0, B3_DERIVE_KEY_MATERIAL);
    b3_root_output(&root, out, out_len);
}

/* ---------------------------------------------------------------------- */
/* The plot, following the paper's stages.                                 */
/* ---------------------------------------------------------------------- */

#define OR_BUCKET_BITS 24
#define OR_NBUCKETS (1u << OR_BUCKET_BITS)

typedef struct {
    uint32_t nonce_a;
    uint32_t nonce_b;
    uint64_t hash2;
} or_t2_record;

static uint64_t load_be64(const uint8_t *p) {
    uint64_t x = 0;
    for (int i = 0; i < 8; i++) x = (x << 8) | p[i];
    return x;
}

/* Table-1 hash of one nonce (sec. III-B: little-endian nonce, keyed BLAKE3
 * with the 256-bit plot key).  Returns key64 = first 8 output bytes read
 * big-endian. */
uint64_t or_h1(const uint8_t key[32], uint32_t nonce) {
    uint8_t msg[4], out[8];
    store_le32(msg, nonce);
    or_b3_hash(key, msg, 4, out, 8);
    return load_be64(out);
}

/* Table-2 hash of a matched pair (sec. II-B / III-A: matched Table-1 nonces
 * are hashed into Table-2 records). */
uint64_t or_h2(const uint8_t key[32], uint32_t nonce_a, uint32_t nonce_b) {
    uint8_t msg[8], out[8];
    store_le32(msg, nonce_a);
    store_le32(msg + 4, nonce_b);
    or_b3_hash(key, msg, 8, out, 8);
    return load_be64(out);
}

uint64_t or_default_threshold(uint32_t k) { return (uint64_t)1 << (64 - k); }

/* Stage 1 (sec. III-A, hash generation): key64 of every nonce in [0, 2^k),
 * stored in nonce order. */
void or_hash_table1(const uint8_t key[32], uint32_t k, uint64_t *keys) {
    uint64_t n = (uint64_t)1 << k;
    for (uint64_t i = 0; i < n; i++) keys[i] = or_h1(key, (uint32_t)i);
}

static int rec_less(uint64_t ka, uint32_t na, uint64_t kb, uint32_t nb) {
    return ka < kb || (ka == kb && na < nb);
}

/* Sort stage (sec. III-A: insertion sort by hash value inside one bucket),
 * ties broken by nonce. */
static void insertion_sort_bucket(uint64_t *keys, uint32_t *nonces, uint64_t len) {
    for (uint64_t i = 1; i < len; i++) {
        uint64_t kk = keys[i];
        uint32_t nn = nonces[i];
        uint64_t j = i;
        while (j > 0 && rec_less(kk, nn, keys[j - 1], nonces[j - 1])) {
            keys[j] = keys[j - 1];
            nonces[j] = nonces[j - 1];
            j--;
        }
        keys[j] = kk;
        nonces[j] = nn;
    }
}

/* Bucketing (sec. I-A, III-B: each record goes to the bucket named by the
 * 24-bit hash prefix): count, prefix-sum into offsets[2^24 + 1], then place
 * the records in nonce order. */
static void bucket_place(uint32_t k, const uint64_t *keys_nonce_order, uint64_t *t1_keys,
                         uint32_t *t1_nonces, uint32_t *offsets) {
    uint64_t n = (uint64_t)1 << k;
    uint32_t *cursor = (uint32_t *)calloc(OR_NBUCKETS, sizeof(uint32_t));
    for (uint64_t i = 0; i < n; i++) cursor[keys_nonce_order[i] >> 40]++;
    uint64_t run = 0;
    for (uint32_t b = 0; b < OR_NBUCKETS; b++) {
        uint32_t c = cursor[b];
        offsets[b] = (uint32_t)run;
        cursor[b] = (uint32_t)run;
        run += c;
    }
    offsets[OR_NBUCKETS] = (uint32_t)run;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t b = (uint32_t)(keys_nonce_order[i] >> 40);
        uint32_t pos = cursor[b]++;
        t1_keys[pos] = keys_nonce_order[i];
        t1_nonces[pos] = (uint32_t)i;
    }
    free(cursor);
}

/* Bucket then sort every bucket: the canonical Table 1 and its bucket
 * offsets (offsets[b] = index of the first record of bucket b). */
void or_bucket_sort(uint32_t k, const uint64_t *keys_nonce_order, uint64_t *t1_keys,
                    uint32_t *t1_nonces, uint32_t *offsets) {
    bucket_place(k, keys_nonce_order, t1_keys, t1_nonces, offsets);
    for (uint32_t b = 0; b < OR_NBUCKETS; b++)
        insertion_sort_bucket(t1_keys + offsets[b], t1_nonces + offsets[b],
                              (uint64_t)offsets[b + 1] - offsets[b]);
}

/* Match stage for buckets [b0, b1) (sec. II-B, III-A): every pair i < j in
 * one bucket whose key distance is below T.  Because the bucket is sorted
 * the scan from i stops at the first j that fails.  Writes at most cap
 * records into out (out may be NULL), returns the full count. */
static uint64_t match_buckets(const uint8_t key[32], uint64_t T, const uint64_t *t1_keys,
                              const uint32_t *t1_nonces, const uint32_t *offsets, uint32_t b0,
                              uint32_t b1, or_t2_record *out, uint64_t cap) {
    uint64_t count = 0;
    for (uint32_t b = b0; b < b1; b++) {
        for (uint64_t i = offsets[b]; i < offsets[b + 1]; i++) {
            for (uint64_t j = i + 1; j < offsets[b + 1] && t1_keys[j] - t1_keys[i] < T; j++) {
                if (out && count < cap) {
                    out[count].nonce_a = t1_nonces[i];
                    out[count].nonce_b = t1_nonces[j];
                    out[count].hash2 = or_h2(key, t1_nonces[i], t1_nonces[j]);
                }
                count++;
            }
        }
    }
    return count;
}

/* Table 2 from a canonical Table 1.  Returns |T2|; writes min(|T2|, cap). */
uint64_t or_match_table2(const uint8_t key[32], uint64_t T, const uint64_t *t1_keys,
                         const uint32_t *t1_nonces, const uint32_t *offsets, or_t2_record *out,
                         uint64_t cap) {
    return match_buckets(key, T, t1_keys, t1_nonces, offsets, 0, OR_NBUCKETS, out, cap);
}

/* Whole plot: hash -> bucket -> sort -> match.  keys_scratch holds the
 * nonce-order hashes ([2^k]). */
uint64_t or_plot(const uint8_t key[32], uint32_t k, uint64_t T, uint64_t *keys_scratch,
                 uint64_t *t1_keys, uint32_t *t1_nonces, uint32_t *offsets, or_t2_record *out,
                 uint64_t cap) {
    or_hash_table1(key, k, keys_scratch);
    or_bucket_sort(k, keys_scratch, t1_keys, t1_nonces, offsets);
    return or_match_table2(key, T, t1_keys, t1_nonces, offsets, out, cap);
}

/* ---------------------------------------------------------------------- */
/* The same stages split over threads (nonce ranges for the hash, bucket   */
/* ranges for sort and match).  The per-item code is the plain code above; */
/* only the loop bounds are divided.  Used for the CPU baseline and to     */
/* check large k within a test's time.                                     */
/* ---------------------------------------------------------------------- */

typedef struct {
    const uint8_t *key;
    uint64_t lo, hi;
    uint64_t *keys;
} h1_job;

static void *h1_worker(void *arg) {
    h1_job *j = (h1_job *)arg;
    for (uint64_t i = j->lo; i < j->hi; i++) j->keys[i] = or_h1(j->key, (uint32_t)i);
    return NULL;
}

void or_hash_table1_mt(const uint8_t key[32], uint32_t k, uint64_t *keys, int nthreads) {
    uint64_t n = (uint64_t)1 << k;
    if (nthreads < 1) nthreads = 1;
    pthread_t th[256];
    h1_job jobs[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; t++) {
        jobs[t].key = key;
        jobs[t].lo = n * t / nthreads;
        jobs[t].hi = n * (t + 1) / nthreads;
        jobs[t].keys = keys;
        pthread_create(&th[t], NULL, h1_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
}

typedef struct {
    uint32_t b0, b1;
    uint64_t *t1_keys;
    uint32_t *t1_nonces;
    const uint32_t *offsets;
} sort_job;

static void *sort_worker(void *arg) {
    sort_job *j = (sort_job *)arg;
    for (uint32_t b = j->b0; b < j->b1; b++)
        insertion_sort_bucket(j->t1_keys + j->offsets[b], j->t1_nonces + j->offsets[b],
                              (uint64_t)j->offsets[b + 1] - j->offsets[b]);
    return NULL;
}

void or_bucket_sort_mt(uint32_t k, const uint64_t *keys_nonce_order, uint64_t *t1_keys,
                       uint32_t *t1_nonces, uint32_t *offsets, int nthreads) {
    bucket_place(k, keys_nonce_order, t1_keys, t1_nonces, offsets);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    sort_job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t].b0 = (uint32_t)((uint64_t)OR_NBUCKETS * t / nthreads);
        jobs[t].b1 = (uint32_t)((uint64_t)OR_NBUCKETS * (t + 1) / nthreads);
        jobs[t].t1_keys = t1_keys;
        jobs[t].t1_nonces = t1_nonces;
        jobs[t].offsets = offsets;
        pthread_create(&th[t], NULL, sort_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
}

typedef struct {
    const uint8_t *key;
    uint64_t T;
    const uint64_t *t1_keys;
    const uint32_t *t1_nonces;
    const uint32_t *offsets;
    uint32_t b0, b1;
    or_t2_record *out;
    uint64_t cap;
    uint64_t count;
} match_job;

static void *match_worker(void *arg) {
    match_job *j = (match_job *)arg;
    j->count = match_buckets(j->key, j->T, j->t1_keys, j->t1_nonces, j->offsets, j->b0, j->b1,
                             j->out, j->cap);
    return NULL;
}

/* Two passes: count per bucket range, then write each range at its prefix. */
uint64_t or_match_table2_mt(const uint8_t key[32], uint64_t T, const uint64_t *t1_keys,
                            const uint32_t *t1_nonces, const uint32_t *offsets,
                            or_t2_record *out, uint64_t cap, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    match_job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t].key = key;
        jobs[t].T = T;
        jobs[t].t1_keys = t1_keys;
        jobs[t].t1_nonces = t1_nonces;
        jobs[t].offsets = offsets;
        jobs[t].b0 = (uint32_t)((uint64_t)OR_NBUCKETS * t / nthreads);
        jobs[t].b1 = (uint32_t)((uint64_t)OR_NBUCKETS * (t + 1) / nthreads);
        jobs[t].out = NULL;
        jobs[t].cap = 0;
        pthread_create(&th[t], NULL, match_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    uint64_t base = 0;
    for (int t = 0; t < nthreads; t++) {
        uint64_t c = jobs[t].count;
        jobs[t].out = out ? out + (base < cap ? base : cap) : NULL;
        jobs[t].cap = base < cap ? cap - base : 0;
        base += c;
    }
    if (out && cap > 0) {
        for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, match_worker, &jobs[t]);
        for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    }
    return base;
}

/* ---------------------------------------------------------------------- */
/* Sampled buckets for sizes whose full tables do not fit the host: hash   */
/* every nonce, keep only records whose bucket is in the sorted list       */
/* buckets[0..nb), then bucket, sort and match those buckets exactly as    */
/* above.  The outputs are the slices of the full Table 1 and Table 2 that */
/* belong to the listed buckets, in bucket order.                          */
/* ---------------------------------------------------------------------- */

typedef struct {
    const uint8_t *key;
    uint64_t lo, hi;
    const uint8_t *bitmap;
    uint64_t *keys;
    uint32_t *nonces;
    uint64_t len, cap;
} sample_job;

static void *sample_worker(void *arg) {
    sample_job *j = (sample_job *)arg;
    j->len = 0;
    j->cap = 1024;
    j->keys = (uint64_t *)malloc(j->cap * sizeof(uint64_t));
    j->nonces = (uint32_t *)malloc(j->cap * sizeof(uint32_t));
    for (uint64_t i = j->lo; i < j->hi; i++) {
        uint64_t h = or_h1(j->key, (uint32_t)i);
        uint32_t b = (uint32_t)(h >> 40);
        if (j->bitmap[b >> 3] & (1u << (b & 7))) {
            if (j->len == j->cap) {
                j->cap *= 2;
                j->keys = (uint64_t *)realloc(j->keys, j->cap * sizeof(uint64_t));
                j->nonces = (uint32_t *)realloc(j->nonces, j->cap * sizeof(uint32_t));
            }
            j->keys[j->len] = h;
            j->nonces[j->len] = (uint32_t)i;
            j->len++;
        }
    }
    return NULL;
}

/* Returns 0 on success, -1 if an output capacity is too small (then
 * *t1_len / *t2_len still hold the sizes needed).  bucket_counts[i] and
 * pair_counts[i] are per listed bucket. */
int or_sample_buckets(const uint8_t key[32], uint32_t k, uint64_t T, const uint32_t *buckets,
                      uint32_t nb, int nthreads, uint64_t *t1_keys, uint32_t *t1_nonces,
                      uint64_t t1_cap, uint32_t *bucket_counts, uint64_t *t1_len,
                      or_t2_record *t2, uint64_t t2_cap, uint64_t *pair_counts,
                      uint64_t *t2_len) {
    uint64_t n = (uint64_t)1 << k;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    uint8_t *bitmap = (uint8_t *)calloc(OR_NBUCKETS / 8, 1);
    for (uint32_t i = 0; i < nb; i++) bitmap[buckets[i] >> 3] |= (uint8_t)(1u << (buckets[i] & 7));
    pthread_t th[256];
    sample_job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t].key = key;
        jobs[t].lo = n * t / nthreads;
        jobs[t].hi = n * (t + 1) / nthreads;
        jobs[t].bitmap = bitmap;
        pthread_create(&th[t], NULL, sample_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(bitmap);

    /* Per listed bucket: count, prefix, place (threads joined in nonce-range
     * order, so placement is in nonce order), then sort. */
    uint64_t total = 0;
    for (int t = 0; t < nthreads; t++) total += jobs[t].len;
    *t1_len = total;
    uint32_t *cursor = (uint32_t *)calloc(nb + 1, sizeof(uint32_t));
    uint32_t *start = (uint32_t *)calloc(nb + 1, sizeof(uint32_t));
    for (int t = 0; t < nthreads; t++)
        for (uint64_t i = 0; i < jobs[t].len; i++) {
            uint32_t b = (uint32_t)(jobs[t].keys[i] >> 40);
            uint32_t lo = 0, hi = nb; /* position of b in the sorted list */
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) / 2;
                if (buckets[mid] <= b) lo = mid; else hi = mid;
            }
            cursor[lo]++;
        }
    uint64_t run = 0;
    for (uint32_t i = 0; i < nb; i++) {
        bucket_counts[i] = cursor[i];
        start[i] = (uint32_t)run;
        run += cursor[i];
        cursor[i] = start[i];
    }
    start[nb] = (uint32_t)run;
    int status = 0;
    if (total > t1_cap) {
        status = -1;
    } else {
        for (int t = 0; t < nthreads; t++)
            for (uint64_t i = 0; i < jobs[t].len; i++) {
                uint32_t b = (uint32_t)(jobs[t].keys[i] >> 40);
                uint32_t lo = 0, hi = nb;
                while (hi - lo > 1) {
                    uint32_t mid = (lo + hi) / 2;
                    if (buckets[mid] <= b) lo = mid; else hi = mid;
                }
                uint32_t pos = cursor[lo]++;
                t1_keys[pos] = jobs[t].keys[i];
                t1_nonces[pos] = jobs[t].nonces[i];
            }
        for (uint32_t i = 0; i < nb; i++)
            insertion_sort_bucket(t1_keys + start[i], t1_nonces + start[i],
                                  (uint64_t)start[i + 1] - start[i]);
        uint64_t pairs = 0;
        for (uint32_t i = 0; i < nb; i++) {
            /* start[] doubles as a bucket-offset array over the listed buckets */
            uint64_t c = match_buckets(key, T, t1_keys, t1_nonces, start, i, i + 1,
                                       t2 ? t2 + (pairs < t2_cap ? pairs : t2_cap) : NULL,
                                       pairs < t2_cap ? t2_cap - pairs : 0);
            pair_counts[i] = c;
            pairs += c;
        }
        *t2_len = pairs;
        if (pairs > t2_cap) status = -1;
    }
    for (int t = 0; t < nthreads; t++) {
        free(jobs[t].keys);
        free(jobs[t].nonces);
    }
    free(cursor);
    free(start);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Timing of the plain single-threaded stages (CPU baseline).             */
/* ---------------------------------------------------------------------- */

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + ts.tv_nsec * 1e-9;
}

/* Runs the plot with nthreads (1 = the plain single-threaded oracle) and
 * reports per-stage wall seconds: secs[0] hash, secs[1] bucket+sort,
 * secs[2] match + Table-2 hash.  Returns |T2|. */
uint64_t or_plot_timed(const uint8_t key[32], uint32_t k, uint64_t T, uint64_t *keys_scratch,
                       uint64_t *t1_keys, uint32_t *t1_nonces, uint32_t *offsets,
                       or_t2_record *out, uint64_t cap, int nthreads, double secs[3]) {
    double t0 = now_s();
    if (nthreads <= 1) or_hash_table1(key, k, keys_scratch);
    else or_hash_table1_mt(key, k, keys_scratch, nthreads);
    double t1 = now_s();
    if (nthreads <= 1) or_bucket_sort(k, keys_scratch, t1_keys, t1_nonces, offsets);
    else or_bucket_sort_mt(k, keys_scratch, t1_keys, t1_nonces, offsets, nthreads);
    double t2 = now_s();
    uint64_t c = nthreads <= 1
                     ? or_match_table2(key, T, t1_keys, t1_nonces, offsets, out, cap)
                     : or_match_table2_mt(key, T, t1_keys, t1_nonces, offsets, out, cap, nthreads);
    double t3 = now_s();
    secs[0] = t1 - t0;
    secs[1] = t2 - t1;
    secs[2] = t3 - t2;
    return c;
}
