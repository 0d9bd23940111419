// Kernels of the index build (quantisation, covariance, eigendecomposition,
// basis, projection, keys) and of the radix sort.
#pragma once

#include "common.hpp"

namespace sfc {

// ---- byte quantisation (vmin/vmax over known voxels, FP32 scale)
// params: float[3] = {vmin, scale, vmax} on the device; part: device
// scratch of 2 * kQuantBlocks uint32 (per-block partial ranges)
constexpr int kQuantBlocks = 1024;
sfc_status launch_quantize(const float* vol, const uint8_t* mask, const Grid& g, uint8_t* xq,
                           float* params, uint32_t* part, hipStream_t st);
// Order-free u64 checksum of the byte codes of the known voxels into *out
// (device), which it clears first.
sfc_status launch_code_checksum(const uint8_t* xq, const uint8_t* mask, int64_t nvox, int C,
                                uint64_t* out, hipStream_t st);

// ---- covariance sums over the strided subsample of dictionary ranks
// elem_off[e] = (voxel offset of pixel e/C) * C + e%C relative to centre*C
// Xt: [P][nsp4] u32, 4 samples per word; nsp4 = ceil(nsub/4)
sfc_status launch_gather_samples(const uint8_t* xq, const uint32_t* dict, int64_t stride,
                                 int64_t nsub, const int32_t* elem_off, int P, int C,
                                 uint32_t* Xt, int64_t nsp4, hipStream_t st);
// sum[e] (u64) and gram[e][f] (u64, full P x P) accumulated; both pre-zeroed
sfc_status launch_gram(const uint32_t* Xt, int P, int64_t nsp4, uint64_t* sum, uint64_t* gram,
                       hipStream_t st);

// ---- per-subset covariance matrix, Jacobi eigensolver and int8 basis
// A: [S][mmax*mmax] doubles; elems: [S][mmax] element ids; m: [S]
sfc_status launch_cov_matrix(const uint64_t* sum, const uint64_t* gram, int64_t nsub, int P,
                             const int32_t* elems, const int32_t* m, int S, int mmax, double* A,
                             hipStream_t st);
// Eigenvectors into V, eigenvalues on A's diagonal; sweeps[S] (int32).
// scratch: jacobi_scratch_bytes(S, mmax) bytes of device memory.
size_t jacobi_scratch_bytes(int S, int mmax);
sfc_status launch_jacobi(double* A, double* V, void* scratch, const int32_t* m, int S, int mmax,
                         int32_t* sweeps, hipStream_t st);
// ---- sort of key arrays (allocates and frees its scratch; synchronizes st)
// narr arrays of n (key, id) pairs, keys [narr][W64][n] (word 0 most
// significant), ids [narr][n]: each array by (key, position), stable, over
// the key bits below nbits.
sfc_status sort_key_arrays(uint64_t* keys, uint32_t* ids, int64_t n, int W64, int narr,
                           int nbits, hipStream_t st);

// int8 basis [S][mmax][D] (row-major per subset) from A/V
sfc_status launch_basis(const double* A, const double* V, const int32_t* m, int S, int mmax,
                        int D, int8_t* basis, hipStream_t st);

}  // namespace sfc
