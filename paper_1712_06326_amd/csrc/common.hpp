// Internal declarations shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/sfcinpaint.h"

namespace sfc {

constexpr int kMaxDims = 3;
constexpr int kMaxChannels = 16;
constexpr int kMaxKeyWords = 4;   // D*b <= 256 bits
constexpr int kMaxD = 32;         // reduced dimension
constexpr int kMaxSubsetElems = 518;

// Geometry as the kernels see it: spatial strides and the interior box of
// valid patch centres.
struct Grid {
    int nd;
    int C;
    int K;
    int h;            // (K-1)/2
    int Kd;           // K^nd
    int rows;         // K^(nd-1): patch rows along the fastest axis
    int64_t shape[kMaxDims];
    int64_t stride[kMaxDims];
    int64_t nvox;
};

Grid make_grid(const sfc_geometry* g, int K);

// thread-local error reporting used by the ABI layer
void set_error(const std::string& msg);
void clear_error();

struct Status {
    sfc_status code = SFC_OK;
    bool ok() const { return code == SFC_OK; }
};

sfc_status fail(sfc_status code, const std::string& msg);
sfc_status check_hip(hipError_t e, const char* what);

#define SFC_HIP(call)                                                       \
    do {                                                                    \
        hipError_t e__ = (call);                                            \
        if (e__ != hipSuccess) return ::sfc::check_hip(e__, #call);         \
    } while (0)

#define SFC_TRY(call)                                                       \
    do {                                                                    \
        sfc_status s__ = (call);                                            \
        if (s__ != SFC_OK) return s__;                                      \
    } while (0)

// ------------------------------------------------------------ kernels API
// (all enqueue on `st`, return SFC_OK or SFC_EDEVICE on a launch error)

// flags[v] = 1 for fill-front voxels.
sfc_status launch_front_flags(const uint8_t* mask, const Grid& g, uint8_t* flags, hipStream_t st);
// Ascending indices i with flags[i] != 0. out64 or out32 (one non-null);
// count_dev receives the total (int64). scratch: see compact_scratch_bytes.
size_t compact_scratch_bytes(int64_t n);
sfc_status launch_compact(const uint8_t* flags, int64_t n, int64_t* out64, uint32_t* out32,
                          int64_t cap, int64_t* count_dev, void* scratch, hipStream_t st);
sfc_status launch_extract(const float* vol, const uint8_t* mask, const Grid& g,
                          const int64_t* centres, int64_t Q, float* t, uint8_t* m,
                          hipStream_t st);
// valid[v] = 1 iff the K^nd box at v is inside and fully known; tmp: nvox bytes
sfc_status launch_valid_centres(const uint8_t* mask, const Grid& g, uint8_t* valid,
                                uint8_t* tmp, hipStream_t st);
sfc_status launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st);
sfc_status launch_zero_f32(float* p, int64_t n, hipStream_t st);
// out[i] = in[i] for i < n, 0 for n <= i < npad
sfc_status launch_pad_f32(const float* in, int64_t n, int64_t npad, float* out, hipStream_t st);
sfc_status launch_u32_to_i64(const uint32_t* in, int64_t* out, int64_t n, hipStream_t st);

// float32 full scan: best[q] = min over valid centres of (cost bits << 32 | id)
struct ScanArgs {
    const float* vol;
    const uint8_t* valid;
    const float* t;            // [scan_qpad(Q), K^nd, C], rows beyond Q zero
    const uint32_t* rowmask;   // [rows, scan_qpad(Q)] bit dx set when (row, dx) is known
    int64_t Q;
    uint64_t* best;            // [Q], pre-filled with ~0
    int query_block;           // 0 = default
    int variant;               // scan shape variant (0 = default)
    const uint32_t* spans;     // dictionary spans (null: whole lines)
    int64_t n_spans;
    int norm;                  // 0: L2 cost, 1: L1 cost (default tile shape)
};
sfc_status launch_pack_rowmask(const uint8_t* m, const Grid& g, int64_t Q, uint32_t* rowmask,
                               hipStream_t st);
sfc_status launch_scan_fp32(const Grid& g, const ScanArgs& a, hipStream_t st);
int64_t scan_qpad(int64_t Q);  // row-mask query stride
// spans of 8 consecutive line positions (the scan's tiling of the interior)
// that hold at least one dictionary centre: slots, flags, compacted list
int64_t scan_span_slots(const Grid& g);
sfc_status launch_span_flags(const Grid& g, const uint8_t* valid, uint8_t* flags, hipStream_t st);
int scan_variants(int nd, int K, int C);
sfc_status launch_unpack_best(const uint64_t* best, int64_t Q, int64_t* id, float* cost,
                              hipStream_t st);

}  // namespace sfc
