// Keyed BLAKE3 of one short message, one lane per message, for gfx950.
//
// The plotter hashes 4-byte nonces (Table 1) and 8-byte nonce pairs
// (Table 2) with keyed BLAKE3 (paper sec. I-A, I-B, III-B).  A message of
// at most 64 bytes is a single chunk with a single block, so its hash is one
// compression (BLAKE3 specification sec. 2.2) of the zero-padded block with
// the key words as chaining value, counter 0, block length = message bytes,
// flags CHUNK_START | CHUNK_END | ROOT | KEYED_HASH; the digest is the first
// output words, out[i] = v[i] ^ v[i + 8].
//
// Design for CDNA4: the key is a kernel argument (SGPRs), so everything that
// depends on the key alone -- three of the four first-round column G's and
// the key half of the first one -- is uniform and the compiler runs it on
// the scalar unit; the message words other than m0/m1 are literal zeros and
// fold away; only v0, v1, v8 and v9 of the last round are live, so the dead
// tail of the last round is removed.  What remains per lane is 32-bit
// add/xor/rotate on the VALU (rotate = v_alignbit_b32 or a byte permute).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vxd {

struct Key {
    uint32_t w[8];  // the 32-byte plot key as eight little-endian words
};

// BLAKE3 IV words 0..3 (the SHA-256 initial value), which seed v[8..11].
constexpr uint32_t kIV0 = 0x6A09E667u;
constexpr uint32_t kIV1 = 0xBB67AE85u;
constexpr uint32_t kIV2 = 0x3C6EF372u;
constexpr uint32_t kIV3 = 0xA54FF53Au;

// Flags of a keyed root chunk made of one block.
constexpr uint32_t kFlagChunkStart = 1u;
constexpr uint32_t kFlagChunkEnd = 2u;
constexpr uint32_t kFlagRoot = 8u;
constexpr uint32_t kFlagKeyedHash = 16u;
constexpr uint32_t kKeyedSingleBlock = kFlagChunkStart | kFlagChunkEnd | kFlagRoot | kFlagKeyedHash;

// Message word order per round: round 0 takes m[0..15] in order and each
// later round applies the specification's fixed permutation to the previous
// round's order.  Built at compile time so every index below is a constant.
struct RoundOrder {
    int w[7][16];
};

constexpr RoundOrder make_round_order() {
    constexpr int perm[16] = {2, 6, 3, 10, 7, 0, 4, 13, 1, 11, 12, 5, 9, 14, 15, 8};
    RoundOrder o{};
    for (int i = 0; i < 16; ++i) o.w[0][i] = i;
    for (int r = 1; r < 7; ++r)
        for (int i = 0; i < 16; ++i) o.w[r][i] = o.w[r - 1][perm[i]];
    return o;
}

constexpr RoundOrder kOrder = make_round_order();

__device__ __forceinline__ uint32_t rotr32(uint32_t x, uint32_t n) {
    return __builtin_amdgcn_alignbit(x, x, n);
}

#define VXD_G(a, b, c, d, mx, my)      \
    do {                               \
        a = a + b + (mx);              \
        d = rotr32(d ^ a, 16);         \
        c = c + d;                     \
        b = rotr32(b ^ c, 12);         \
        a = a + b + (my);              \
        d = rotr32(d ^ a, 8);          \
        c = c + d;                     \
        b = rotr32(b ^ c, 7);          \
    } while (0)

// Message word `slot` of round R for a message whose only non-zero words
// are m0 and m1.
template <int R, int Slot>
__device__ __forceinline__ uint32_t msg(uint32_t m0, uint32_t m1) {
    constexpr int idx = kOrder.w[R][Slot];
    return idx == 0 ? m0 : (idx == 1 ? m1 : 0u);
}

template <int R>
__device__ __forceinline__ void round_fn(uint32_t &v0, uint32_t &v1, uint32_t &v2, uint32_t &v3,
                                         uint32_t &v4, uint32_t &v5, uint32_t &v6, uint32_t &v7,
                                         uint32_t &v8, uint32_t &v9, uint32_t &v10,
                                         uint32_t &v11, uint32_t &v12, uint32_t &v13,
                                         uint32_t &v14, uint32_t &v15, uint32_t m0,
                                         uint32_t m1) {
    VXD_G(v0, v4, v8, v12, (msg<R, 0>(m0, m1)), (msg<R, 1>(m0, m1)));
    VXD_G(v1, v5, v9, v13, (msg<R, 2>(m0, m1)), (msg<R, 3>(m0, m1)));
    VXD_G(v2, v6, v10, v14, (msg<R, 4>(m0, m1)), (msg<R, 5>(m0, m1)));
    VXD_G(v3, v7, v11, v15, (msg<R, 6>(m0, m1)), (msg<R, 7>(m0, m1)));
    VXD_G(v0, v5, v10, v15, (msg<R, 8>(m0, m1)), (msg<R, 9>(m0, m1)));
    VXD_G(v1, v6, v11, v12, (msg<R, 10>(m0, m1)), (msg<R, 11>(m0, m1)));
    VXD_G(v2, v7, v8, v13, (msg<R, 12>(m0, m1)), (msg<R, 13>(m0, m1)));
    VXD_G(v3, v4, v9, v14, (msg<R, 14>(m0, m1)), (msg<R, 15>(m0, m1)));
}

// key64 of a message of `block_len` (<= 8) bytes held in m0 (bytes 0..3,
// little-endian) and m1 (bytes 4..7): the first 8 digest bytes read
// big-endian, so that numeric order is byte order.
__device__ __forceinline__ uint64_t keyed_hash64(const Key &k, uint32_t m0, uint32_t m1,
                                                 uint32_t block_len) {
    uint32_t v0 = k.w[0], v1 = k.w[1], v2 = k.w[2], v3 = k.w[3];
    uint32_t v4 = k.w[4], v5 = k.w[5], v6 = k.w[6], v7 = k.w[7];
    uint32_t v8 = kIV0, v9 = kIV1, v10 = kIV2, v11 = kIV3;
    uint32_t v12 = 0u, v13 = 0u, v14 = block_len, v15 = kKeyedSingleBlock;
    round_fn<0>(v0, v1, v2, v3, v4, v5, v6, v7, v8, v9, v10, v11, v12, v13, v14, v15, m0, m1);
    round_fn<1>(v0, v1, v2, v3, v4, v5, v6, v7, v8, v9, v10, v11, v12, v13, v14, v15, m0, m1);
    round_fn<2>(v0, v1, v2, v3, v4, v5, v6, v7, v8, v9, v10, v11, v12, v13, v14, v15, m0, m1);
    round_fn<3>(v0, v1, v2, v3, v4, v5, v6, v7, v8, v9, v10, v11, v12, v13, v14, v15, m0, m1);
    round_fn<4>(v0, v1, v2, v3, v4, v5, v6, v7, v8, v9, v10, v11, v12, v13, v14, v15, m0, m1);
    round_fn<5>(v0, v1, v2, v3, v4, v5, v6, v7, v8, v9, v10, v11, v12, v13, v14, v15, m0, m1);
    round_fn<6>(v0, v1, v2, v3, v4, v5, v6, v7, v8, v9, v10, v11, v12, v13, v14, v15, m0, m1);
    const uint32_t o0 = v0 ^ v8;
    const uint32_t o1 = v1 ^ v9;
    return ((uint64_t)__builtin_bswap32(o0) << 32) | (uint64_t)__builtin_bswap32(o1);
}

// Table-1 hash: 4-byte little-endian nonce.
__device__ __forceinline__ uint64_t h1(const Key &k, uint32_t nonce) {
    return keyed_hash64(k, nonce, 0u, 4u);
}

// Table-2 hash: LE32(a) || LE32(b).
__device__ __forceinline__ uint64_t h2(const Key &k, uint32_t a, uint32_t b) {
    return keyed_hash64(k, a, b, 8u);
}

#undef VXD_G

}  // namespace vxd
