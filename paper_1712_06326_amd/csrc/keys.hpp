// Device helpers shared by the key kernel of the build and the query
// prologue: curve keys of a grid cell.
#pragma once

#include "common.hpp"

namespace sfc {

// Hilbert index of a point by J. Skilling's transpose method ("Programming
// the Hilbert curve", AIP Conf. Proc. 707, 2004), in place on X[0..D).
__device__ __forceinline__ void hilbert_axes_to_transpose(uint32_t* X, int D, int b) {
    const uint32_t top = 1u << (b - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t low = q - 1;
        for (int i = 0; i < D; i++) {
            if (X[i] & q) {
                X[0] ^= low;
            } else {
                const uint32_t sw = (X[0] ^ X[i]) & low;
                X[0] ^= sw;
                X[i] ^= sw;
            }
        }
    }
    for (int i = 1; i < D; i++) X[i] ^= X[i - 1];
    uint32_t flip = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (X[D - 1] & q) flip ^= q - 1;
    for (int i = 0; i < D; i++) X[i] ^= flip;
}

// Bit l of coordinate d lands at bit l*D + (D-1-d) of the D*b-bit key:
// level by level from the top, dim 0 first. Word 0 is the most significant.
// Each level's D bits are gathered into one group and placed at once.
__device__ __forceinline__ void interleave_words(const uint32_t* v, int D, int b, int W64, uint64_t* w) {
    for (int i = 0; i < W64; i++) w[i] = 0;
    for (int l = 0; l < b; l++) {
        uint64_t grp = 0;
        for (int d = 0; d < D; d++) grp = (grp << 1) | ((v[d] >> l) & 1u);
        const int pos = l * D;
        const int wi = W64 - 1 - (pos >> 6), sh = pos & 63;
        w[wi] |= grp << sh;
        if (sh + D > 64) w[wi - 1] |= grp >> (64 - sh);
    }
}

}  // namespace sfc
