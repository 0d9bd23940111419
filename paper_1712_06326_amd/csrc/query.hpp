// Arguments of the index-query kernels (Fig. 1 b-d).
#pragma once

#include "common.hpp"

namespace sfc {

struct QueryIndexView {
    int nd, K, C, Kd, rows, h;
    int64_t shape[kMaxDims], stride[kMaxDims];
    int S, D, L, b, curve, W64, window, mmax;
    int64_t R, n, nsub;
    const float* qparams;      // device {vmin, scale}
    const int32_t* npix;       // [S]
    const int32_t* pix;        // [S][Kd]
    const int8_t* basis;       // [S][mmax][D]
    const int64_t* wtw;        // [S][D][D] = W^T W (exact)
    const int64_t* ws;         // [S][D] = W^T S, S the subsample sums (exact)
    const uint64_t* smask;     // [S][ceil(Kd/64)] pixel bit mask of each subset
    const uint64_t* sum;       // [P] subsample sums
    const int64_t* lo;         // [S][D]
    const int64_t* span;       // [S]
    const uint64_t* keys;      // [S][L][W64][n]
    const uint32_t* ids;       // [S][L][n]
};

// subset, real coordinates [Q][D] and keys [Q][L][W64] of each query; with
// rowmask non-null also the rescoring's row masks [rows][qpad] (bit dx of
// row r: pixel r*K + dx known), written for queries < Q only; with qbest
// and qticket non-null (both or neither) and Q <= 256 also qbest[q] =
// all-ones and qticket[q] = 0, the split rescoring's starting words
sfc_status launch_query_prologue(const QueryIndexView& v, const float* t, const uint8_t* m,
                                 int64_t Q, int32_t* qsub, double* qcoords, uint64_t* qkeys,
                                 uint32_t* rowmask, int64_t qpad, uint64_t* qbest,
                                 int32_t* qticket, hipStream_t st);
// window start per (query, curve): wstart [Q][L]
sfc_status launch_query_search(const QueryIndexView& v, const int32_t* qsub,
                               const uint64_t* qkeys, int64_t Q, int64_t* wstart, hipStream_t st);
// candidates = union of windows (sorted unique); best (cost, id) over them
// under norm 0 (L2) or 1 (L1). best_id/best_cost or cand/ncand may be null.
// qbest/qticket [Q]: as cleared by the prologue, or null (then a handful of
// queries is not split over workgroups). apply (the fill loop's lone target,
// Q = 1, split form only): the answer is also applied to the loop's state.
struct LoopApply;
sfc_status launch_query_rescore(const QueryIndexView& v, const float* vol, const float* t,
                                const uint32_t* rowmask, int64_t qpad, const int32_t* qsub,
                                const int64_t* wstart, int64_t Q, int64_t* best_id,
                                float* best_cost, int64_t* cand, int32_t* ncand, int norm,
                                uint64_t* qbest, int32_t* qticket, const LoopApply* apply,
                                hipStream_t st);

// Exact k-NN query (Section II.D) on curve 0 of each query's subset: the k
// nearest entries by (squared cell distance, id), ids ascending in list
// [Q][k], counts in cnt; thr[q] = 0. overflow (one word, zeroed by the
// caller) is set if a traversal stack would overflow.
sfc_status launch_knn(const QueryIndexView& v, const int32_t* qsub, const double* qcoords,
                      int64_t Q, int k, int mu, uint32_t* list, int32_t* cnt, int32_t* thr,
                      unsigned int* overflow, hipStream_t st);
// list/cnt -> cand int64 [Q][k] padded -1 and ncand [Q] (either may be null)
sfc_status launch_knn_cand(const uint32_t* list, const int32_t* cnt, int64_t Q, int k,
                           int64_t* cand, int32_t* ncand, hipStream_t st);

}  // namespace sfc
