// The handle behind the opaque sfc_index and the host-side entry points of
// the build and query paths.
#pragma once

#include <vector>

#include "common.hpp"

namespace sfc {

sfc_status dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void* p);
// stream-ordered temporaries (freeing one does not wait for other streams)
sfc_status tmp_alloc(void** p, size_t bytes, const char* what, hipStream_t st);
void tmp_free(void* p, hipStream_t st);

// One stream-ordered temporary, freed on its stream at scope exit.
struct TmpBuf {
    hipStream_t st;
    void* ptr = nullptr;
    explicit TmpBuf(hipStream_t s) : st(s) {}
    sfc_status alloc(size_t bytes, const char* what) { return tmp_alloc(&ptr, bytes, what, st); }
    ~TmpBuf() { tmp_free(ptr, st); }
    TmpBuf(const TmpBuf&) = delete;
    TmpBuf& operator=(const TmpBuf&) = delete;
};

// Grow-only device scratch buffer owned by a handle.
struct Scratch {
    void* ptr = nullptr;
    size_t cap = 0;
    sfc_status reserve(size_t bytes, const char* what);
    ~Scratch();
};

// HIP-event timing of a handle's main query kernels (options.timing = 1):
// begin/end bracket one launch on the handle's stream; the events are pooled
// and reused by the next query.
// Events around the timed kernels of the queries made since the times were
// last read (sfc_query_kernel_times clears them); at most kMaxMarks launches
// are kept.
struct KernelTimer {
    static constexpr int kMaxMarks = 4096;
    struct Mark {
        const char* name = nullptr;
        hipEvent_t a = nullptr, b = nullptr;
    };
    std::vector<Mark> marks;
    mutable int used = 0;
    bool on = false;
    bool open = false;   // begin recorded, end pending
    // timing on or off for the next query; unread marks are kept
    void reset(bool enable) { on = enable; }
    sfc_status begin(const char* name, hipStream_t st);
    sfc_status end(hipStream_t st);
    ~KernelTimer();
};

sfc_options resolve_options(const sfc_options* in);
void remember_variant(int nd, int K, int C, int v);
int recalled_variant(int nd, int K, int C);

}  // namespace sfc

struct sfc_index {
    sfc::Grid g{};
    sfc_options opt{};
    hipStream_t st = nullptr;
    int device = -1;                 // the device current when the handle was made
    const float* vol = nullptr;      // borrowed
    uint8_t* valid = nullptr;        // [nvox] 1 = dictionary centre
    uint32_t* dict = nullptr;        // [n] ascending centre ids
    uint32_t* spans = nullptr;       // [n_spans] scan spans holding a centre
    int64_t n_spans = 0;
    int64_t n = 0;

    // ---- SFC multi-index (Section II)
    bool has_sfc = false;
    int S = 0, D = 0, L = 0, b = 0, W64 = 0, mmax = 0;
    int64_t R = 0;
    float vmin = 0.0f, qscale = 0.0f;
    int64_t nsub = 0;
    uint8_t* xq = nullptr;           // [nvox*C] byte codes
    float* qparams = nullptr;        // device {vmin, scale}
    int64_t* sum = nullptr;          // [P] subsample sums (stored as u64)
    int32_t* npix = nullptr;         // [S] pixels per subset
    int32_t* pix = nullptr;          // [S][Kd] pixel offsets, ascending
    int32_t* elems = nullptr;        // [S][mmax] element ids
    int32_t* msz = nullptr;          // [S] element counts
    int32_t* elem_off = nullptr;     // [Pp] element offset relative to centre*C
    int8_t* basis = nullptr;         // [S][mmax][D] int8
    int64_t* wtw = nullptr;          // [S][D][D] W^T W
    int64_t* ws = nullptr;           // [S][D] W^T S (subsample sums)
    uint64_t* smask = nullptr;       // [S][ceil(Kd/64)] subset pixel bit masks
    int64_t* lo = nullptr;           // [S][D]
    int64_t* span = nullptr;         // [S]
    uint64_t* keys = nullptr;        // [S][L][W64][n] sorted key words (one array per word)
    uint32_t* ids = nullptr;         // [S][L][n] sorted ids
    std::vector<int32_t> h_npix, h_pix;
    std::vector<int8_t> h_basis;
    std::vector<int64_t> h_lo, h_span;
    void* proj_w = nullptr;          // bf16 projection weights [tiles*32][Pp]
    uint8_t* mask_copy = nullptr;    // [nvox] the mask at build time
    uint16_t* mfma_B = nullptr;      // reduced-precision scan operand [npad][Kp] bf16
    int Pp = 0;                      // element count padded to 16

    // ---- per-call scratch
    sfc::Scratch rowmask, best, qtmp, tpad, red;
    int64_t last_fallback = 0;
    int64_t last_pass1_tiles = 0, last_pass2_tiles = 0;   // bf16 filter tiles of the last query
    int tuned_variant = 0;           // float32-scan shape chosen by sfc_autotune
    sfc::KernelTimer timer;

    ~sfc_index();
};

namespace sfc {

sfc_status ensure_quantized(sfc_index* ix, const uint8_t* mask);
sfc_status ensure_elem_offsets(sfc_index* ix);
sfc_status check_sfc_args(const sfc_geometry* g, int K, int D, int L, const sfc_options& o);
// What defines a saved index (host copies, in the device layouts); its
// curves follow from these and the dictionary.
struct SavedIndex {
    int64_t nsub = 0;
    float vmin = 0.0f, qscale = 0.0f;
    std::vector<uint64_t> sum;     // [P]
    std::vector<int8_t> basis;     // [S][mmax][D]
    std::vector<int64_t> lo;       // [S][D]
    std::vector<int64_t> span;     // [S]
};
// saved: the statistics and bases of a saved index instead of computing
// them (bases_host unused); its grid must come out the same
sfc_status build_sfc(sfc_index* ix, const uint8_t* mask, int D, int L, const int8_t* bases_host,
                     const SavedIndex* saved = nullptr);
void release_sfc(sfc_index* ix);
// checksum of the byte codes of the known voxels (quantises first if needed)
sfc_status code_checksum(sfc_index* ix, uint64_t* out_host);
// label: the name its launch is timed under
sfc_status query_brute_fp32(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q,
                            uint64_t* best_dev, const char* label = "scan_fp32_kernel");
// The float32 scan on caller buffers: rm [scan_qpad(Q) * rows] u32 row masks,
// tp [scan_qpad(Q) * Kd * C] padded targets, best [Q] packed results. Every
// word of the three is written before it is read.
sfc_status scan_fp32_on(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, uint32_t* rm,
                        float* tp, uint64_t* best, const char* label = "scan_fp32_kernel");
// The scan alone, on row masks, padded targets and a cleared result that
// are already in place.
sfc_status scan_fp32_prepared(sfc_index* ix, int64_t Q, const uint32_t* rm, const float* tp,
                              uint64_t* best, const char* label = "scan_fp32_kernel");
sfc_status query_brute_reduced(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q,
                               sfc_mode mode, int64_t* best_id, float* best_cost);
// forces the reduced-precision scan's list capacity (<= 0: automatic)
void set_list_capacity_override(int32_t cap);
sfc_status query_index(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q,
                       int64_t* best_id, float* best_cost, int64_t* cand, int32_t* ncand);
// The index query on a caller buffer of index_query_bytes(ix, Q) bytes
// (kernel launches only: no allocation, no synchronisation). apply: the
// fill loop's lone target (Q = 1, best answer only), whose answer the
// rescoring's last workgroup also applies to the loop's state.
size_t index_query_bytes(const sfc_index* ix, int64_t Q);
struct LoopApply;
sfc_status query_index_on(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, void* buf,
                          int64_t* best_id, float* best_cost, int64_t* cand, int32_t* ncand,
                          const LoopApply* apply = nullptr);
sfc_status query_coords(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q,
                        int32_t* subset, double* coords);
sfc_status query_knn(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, int k, int mu,
                     int64_t* best_id, float* best_cost, int64_t* cand, int32_t* ncand);

}  // namespace sfc
