// Reduced-precision full scan: exact-integer bf16 MFMA filter + rescoring.
#pragma once

#include "common.hpp"

namespace sfc {

constexpr int kFilterRows = 256;   // queries per filter workgroup (and operand row padding)

struct FilterArgs {
    const uint16_t* A;       // [Kp/32][Qpad][32] bf16 bits (chunk-major), Qpad a multiple of kFilterRows
    const uint16_t* B;       // [Kp/32][npad][32] bf16 bits (chunk-major), npad a multiple of 256
    const int32_t* T2;       // [Qpad]
    int64_t Q, n;
    int Kp;
    const uint32_t* dict;    // dictionary centres by rank
    int32_t* tilemin;        // [Q][ngroups] pass 1: minimum partial Eq per tile group
    const int32_t* thr;      // [Q] pass 2 threshold (-1: the float32 scan answers)
    int32_t* cnt;            // [Q] pass 2 set sizes
    uint32_t* list;          // [Q][cap] pass 2 candidate ids
    const uint64_t* work;    // pass 2 (query tile << 32 | candidate tile)
    int cap;
    int64_t ntiles;          // tiles the launch walks (set by the launcher)
    // filled by plan_filter
    bool drain;              // accumulators drained to int32 (long operands)
    uint64_t drain_mask[2];  // chunks of 32 columns after which to drain
    int bn;                  // candidates per workgroup
    int group;               // candidate tiles per tile-minimum group
    int64_t ctiles, qtiles, ctiles_per_xcd, ngroups;
    int64_t crows;           // rows of the dictionary operand (n rounded up to 256)
    int xq;                  // query-tile groups across the 8 XCDs (1, 2, 4 or 8)
    int64_t all_tiles;       // slots of the XCD-aware order (8 x the largest share)
};

// operand width: per pixel C + 2 columns, padded to a multiple of 32
int64_t mfma_kp(int Kd, int C);
sfc_status plan_filter(int Kd, int C, int64_t Q, int64_t n, FilterArgs* a);
sfc_status launch_dict_operand(const uint8_t* xq, const uint32_t* dict, int64_t n, int64_t npad,
                               const int32_t* elem_off, int Kd, int C, int Kp, uint16_t* B,
                               hipStream_t st);
sfc_status launch_query_operand(const float* t, const uint8_t* m, int64_t Q, int64_t Qpad, int Kd,
                                int C, int Kp, const float* qp, uint16_t* A, int32_t* T2,
                                int32_t* kq, int32_t* flag, hipStream_t st);
// pass 1 of the two-pass filter: per-query minima per tile group
sfc_status launch_filter_minima(FilterArgs a, hipStream_t st);
// thr from the tile minima (two-pass) or from a known upper bound (seeded)
sfc_status launch_threshold(const FilterArgs& a, const int32_t* kq, const int32_t* flag,
                            const float* qp, int32_t* thr, hipStream_t st);
sfc_status launch_seed_threshold(const float* tau, const int32_t* kq, const int32_t* flag,
                                 const float* qp, int64_t Q, int32_t* thr, hipStream_t st);
// pass-2 work list of the two-pass filter
sfc_status launch_select(const FilterArgs& a, uint64_t* work, unsigned long long* nwork,
                         hipStream_t st);
// list every candidate with Eq <= thr: over the work list (nwork >= 0) or
// over all tiles (nwork < 0); clears cnt first
sfc_status launch_filter_list(FilterArgs a, int64_t nwork, hipStream_t st);
// exact rescoring of each query's candidate list; fb[q] = 1 when the list
// overflowed or the threshold was invalid (the float32 scan must answer q)
sfc_status launch_list_rescore(const Grid& g, const float* vol, const float* t,
                               const uint32_t* rowmask, int64_t qpad, const uint32_t* list,
                               const int32_t* cnt, const int32_t* thr, int cap, int64_t Q,
                               int64_t* best_id, float* best_cost, uint8_t* fb, int norm,
                               hipStream_t st);

}  // namespace sfc
