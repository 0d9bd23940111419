// Float32 scan parameters and the batched (many images) scan.
#pragma once

#include "common.hpp"

namespace sfc {

// One image for the float32 scan kernels.
struct ScanParams {
    const float* vol;
    const uint8_t* valid;
    const float* t;          // [qpad][rows][K*C] padded targets
    const uint32_t* rowmask; // [rows][qpad]
    uint64_t* best;          // [Q] packed (cost bits << 32 | id)
    int64_t Q;
    int64_t shape[kMaxDims];
    int64_t stride[kMaxDims];
    int64_t line_len;        // interior extent along the fastest axis
    int64_t tiles_per_line;
    int64_t n_tiles;
    int64_t tiles_per_wg;
    int64_t q_per_wg;
    int64_t qpad;            // row-mask stride (queries padded to the block size)
    int64_t n_chunks, chunks_per_xcd, q_splits;
    int64_t q_group;         // query splits walked over every chunk of a band in turn
    // null: tiles cover whole lines; else the tiles walk this list of spans
    // (8 line positions, index line * spans_per_line + x / 8) that hold a
    // dictionary centre
    const uint32_t* spans;
    int64_t n_spans, spans_per_line;
};

// A batch work item: queries [q0, q1) of one image against its line tiles
// [tl0, tl1).
struct BatchItem {
    int32_t image, pad_;
    int64_t q0, q1, tl0, tl1;
};

// Where one image's queries live in the batch buffers.
struct BatchMeta {
    int64_t Q, qpad;         // queries, and padded to the scan's query block
    int64_t q_off;           // first query (masks, results)
    int64_t t_off;           // first target float
    int64_t tpad_off;        // first padded-target float
    int64_t rm_off;          // first row-mask word
    int32_t C, pad_;
};

bool batch_scan_supported(int K);
int batch_query_block(int shape);
// (QB, NX) of shape set `shape` (0, 1, 2) and the image's tile count
// spans/n_spans: the image's dictionary spans (null: whole lines)
ScanParams batch_image_params(const Grid& g, const float* vol, const uint8_t* valid,
                              const uint32_t* spans, int64_t n_spans, const float* t,
                              const uint32_t* rowmask, uint64_t* best, int64_t Q, int64_t qpad,
                              int shape, int64_t* n_tiles);
sfc_status launch_batch_prep(const float* targets, const uint8_t* masks, const BatchMeta* meta,
                             const int64_t* pad_start, int n_images, int K, int64_t total_pad,
                             float* tpad, uint32_t* rowmask, uint64_t* best, hipStream_t st);
sfc_status launch_batch_scan(int K, int shape, const ScanParams* imgs, const int32_t* img_c,
                             const BatchItem* items, int64_t n_items, unsigned grid,
                             hipStream_t st);

}  // namespace sfc
