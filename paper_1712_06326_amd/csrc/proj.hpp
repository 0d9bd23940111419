// Arguments of the projection and key kernels.
#pragma once

#include "common.hpp"

namespace sfc {

struct ProjArgs {
    const uint8_t* xq;        // quantised volume [nvox*C]
    const uint32_t* dict;     // dictionary centres by rank
    int64_t r0;               // first rank of this chunk
    int64_t cnt;              // patches in this chunk
    const int32_t* elem_off;  // [P] element offset relative to centre*C
    int P, Pk, C;             // elements; Pk = proj_depth(P)
    int run;                  // K*C: contiguous bytes along a patch's innermost axis
    const int8_t* Wt;         // [proj_tiles(ncols)*32][Pk] int8 weights, zero padded
    const int32_t* wsum;      // [proj_tiles(ncols)*32] 128 * (sum of the column's weights)
    int ncols;                // S*D
    int32_t* y;               // [cnt][ystride] or null
    int ystride;
    int32_t* colmin;          // [ncols] or null
    int32_t* colmax;
};

struct KeyArgs {
    const int32_t* y;         // [cnt][ystride]
    int64_t cnt, r0, n;
    int ystride;
    const uint32_t* dict;
    int S, D, L, b, curve, W64;
    int64_t R;
    const int64_t* lo;        // [S][D]
    const int64_t* span;      // [S]
    uint64_t* keys;           // [S][L][W64][n]
    uint32_t* ids;            // [S][L][n]
};

int proj_tiles(int ncols);
// element count padded to the MFMA depth (32)
int proj_depth(int P);
// bytes of the projection weights: int8 [tiles*32][Pk], then int32 [tiles*32]
size_t proj_weight_bytes(int ncols, int P);
// Wt (zeroed beforehand) and its column sums, from the int8 bases
sfc_status launch_weights(const int8_t* basis, const int32_t* elems, const int32_t* msz, int S,
                          int mmax, int D, int P, int ncols, int8_t* Wt, int32_t* wsum,
                          hipStream_t st);
sfc_status launch_init_minmax(int32_t* mn, int32_t* mx, int n, hipStream_t st);
sfc_status launch_projection(const ProjArgs& a, hipStream_t st);
sfc_status launch_span(const int32_t* mn, const int32_t* mx, int S, int D, int64_t* lo,
                       int64_t* span, hipStream_t st);
sfc_status launch_keys(const KeyArgs& a, hipStream_t st);

// ---- radix sort of (multi-word key, id) pairs, stable, ascending
struct SortPlan {
    int n_passes;
    int pass_bits[64];        // bit position (from the key's LSB) of each 8-bit digit
};
// bytes of scratch for `arrays` arrays of n items, W64 words: ping-pong copy + histograms
size_t sort_scratch_bytes(int64_t n, int W64, int arrays);
// OR over items of (key XOR key[0]) for `arrays` consecutive arrays -> varying[arr][W64]
sfc_status launch_varying_bits(const uint64_t* keys, int64_t n, int W64, int arrays,
                               uint64_t* varying, hipStream_t st);
// Sorts `arrays` consecutive arrays (keys [arrays][W64][n], ids [arrays][n])
// with the same digit passes.
sfc_status radix_sort(uint64_t* keys, uint32_t* ids, int64_t n, int W64, int arrays,
                      const SortPlan& plan, void* scratch, hipStream_t st);

}  // namespace sfc
