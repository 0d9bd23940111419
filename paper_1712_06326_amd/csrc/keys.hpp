// Device helpers shared by the key kernel of the build and the query
// prologue: curve keys of a grid cell.
#pragma once

#include "common.hpp"

namespace sfc {

// Hilbert index of a point by J. Skilling's transpose method ("Programming
// the Hilbert curve", AIP Conf. Proc. 707, 2004), in place on X[0..D). The
// loops over axes run to the compile-time bound MD >= D with guards, so X
// stays in registers; the conditional exchanges are written as selects.
template <int MD>
__device__ __forceinline__ void hilbert_axes_to_transpose(uint32_t* X, int D, int b) {
    const uint32_t top = 1u << (b - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t low = q - 1;
#pragma unroll
        for (int i = 0; i < MD; i++) {
            if (i < D) {
                const bool on = (X[i] & q) != 0;
                const uint32_t sw = on ? 0u : ((X[0] ^ X[i]) & low);
                X[0] ^= on ? low : sw;
                X[i] ^= sw;
            }
        }
    }
#pragma unroll
    for (int i = 1; i < MD; i++)
        if (i < D) X[i] ^= X[i - 1];
    uint32_t last = 0;
#pragma unroll
    for (int i = 0; i < MD; i++)
        if (i == D - 1) last = X[i];
    uint32_t flip = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (last & q) flip ^= q - 1;
#pragma unroll
    for (int i = 0; i < MD; i++)
        if (i < D) X[i] ^= flip;
}

// Bit l of coordinate d lands at bit l*D + (D-1-d) of the D*b-bit key:
// level by level from the top, dim 0 first. Word 0 is the most significant.
// 8 x 8 bit-matrix transpose of a 64-bit word, bit 8r + c <-> bit 8c + r
// (swaps of 1x1, 2x2 and 4x4 blocks across the diagonal).
__device__ __forceinline__ uint64_t transpose8x8(uint64_t x) {
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x ^= t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x ^= t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x ^= t ^ (t << 28);
    return x;
}

// The levels enter a 256-bit accumulator from the top level down: each
// shifts it left by D and puts its D bits (dim 0 highest) at the bottom.
// For D = 8 a level is one byte, so the 64-bit word of levels 8j..8j+7 is
// the transpose of the 8 x 8 bit matrix whose row 7 - d is byte j of v[d].
template <int MD>
__device__ __forceinline__ void interleave_words(const uint32_t* v, int D, int b, int W64, uint64_t* w) {
    static_assert(kMaxKeyWords == 4, "the accumulator holds four words");
    if (MD >= 8 && D == 8) {
        const uint32_t keep = b >= 32 ? 0xffffffffu : ((1u << b) - 1u);
        uint64_t a[4];   // a[3] least significant: levels 0..7
#pragma unroll
        for (int j = 0; j < 4; j++) {
            uint64_t x = 0;
#pragma unroll
            for (int d = 0; d < 8; d++)
                x |= (uint64_t)(((v[d] & keep) >> (8 * j)) & 0xffu) << (8 * (7 - d));
            a[3 - j] = transpose8x8(x);
        }
#pragma unroll
        for (int k = 0; k < kMaxKeyWords; k++) {
            const int src = kMaxKeyWords - W64 + k;
            w[k] = src == 0 ? a[0] : src == 1 ? a[1] : src == 2 ? a[2] : a[3];
        }
        return;
    }
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;   // a0 most significant
    const int rs = 64 - D;                     // 1 <= D <= 32
    for (int l = b - 1; l >= 0; l--) {
        uint64_t grp = 0;
#pragma unroll
        for (int d = 0; d < MD; d++)
            if (d < D) grp = (grp << 1) | ((v[d] >> l) & 1u);
        a0 = (a0 << D) | (a1 >> rs);
        a1 = (a1 << D) | (a2 >> rs);
        a2 = (a2 << D) | (a3 >> rs);
        a3 = (a3 << D) | grp;
    }
    // the key's words are the low W64 words of (a0, a1, a2, a3)
#pragma unroll
    for (int k = 0; k < kMaxKeyWords; k++) {
        const int src = kMaxKeyWords - W64 + k;
        w[k] = src == 0 ? a0 : src == 1 ? a1 : src == 2 ? a2 : a3;
    }
}

// Inverse of interleave_words for the Morton order: w holds the key's W64
// words (word 0 most significant) in w[0..W64); bit l*D + (D-1-d) of the key
// is bit l of coordinate d. The words are right-aligned in a 256-bit
// accumulator that shifts right by D per level, lowest level first.
template <int MD>
__device__ __forceinline__ void morton_decode(const uint64_t* w, int D, int b, int W64,
                                              uint32_t* v) {
    static_assert(kMaxKeyWords == 4, "the accumulator holds four words");
    uint64_t a[4];   // a[3] least significant
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int src = W64 - 4 + j;
        a[j] = src == 0 ? w[0] : src == 1 ? w[1] : src == 2 ? w[2] : src == 3 ? w[3] : 0ull;
    }
#pragma unroll
    for (int d = 0; d < MD; d++) v[d] = 0;
    if (MD >= 8 && D == 8) {
        // the transpose is its own inverse: word j's matrix has row 7 - d
        // = byte j of coordinate d
        const uint32_t keep = b >= 32 ? 0xffffffffu : ((1u << b) - 1u);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint64_t x = transpose8x8(a[3 - j]);
#pragma unroll
            for (int d = 0; d < 8; d++) v[d] |= (uint32_t)((x >> (8 * (7 - d))) & 0xffu) << (8 * j);
        }
#pragma unroll
        for (int d = 0; d < 8; d++) v[d] &= keep;
        return;
    }
    const int ls = 64 - D;   // 1 <= D <= 32
    const uint64_t low = (D == 64) ? ~0ull : ((1ull << D) - 1);
    for (int l = 0; l < b; l++) {
        const uint64_t grp = a[3] & low;
#pragma unroll
        for (int d = 0; d < MD; d++)
            if (d < D) v[d] |= (uint32_t)((grp >> (D - 1 - d)) & 1u) << l;
        a[3] = (a[3] >> D) | (a[2] << ls);
        a[2] = (a[2] >> D) | (a[1] << ls);
        a[1] = (a[1] >> D) | (a[0] << ls);
        a[0] >>= D;
    }
}

}  // namespace sfc
