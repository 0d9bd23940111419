// Reduced-precision full scan: exact-integer bf16 MFMA filter + rescoring.
#pragma once

#include "common.hpp"

namespace sfc {

constexpr int kMfmaTile = 128;   // queries and candidates per workgroup tile
constexpr int kDrainK = 960;     // K values between float32 -> integer drains (< 2^24 bound)

struct FilterArgs {
    const uint16_t* A;       // [Qpad][Kp] bf16 bits
    const uint16_t* B;       // [npad][Kp] bf16 bits
    const int32_t* T2;       // [Qpad]
    int64_t Q, n;
    int Kp;
    const uint32_t* dict;    // dictionary centres by rank
    int32_t* eqmin;          // [Q] pass 1 output
    const int32_t* thr;      // [Q] pass 2 threshold
    int32_t* cnt;            // [Q] pass 2 set sizes
    uint32_t* list;          // [Q][cap] pass 2 candidate ids
    int cap;
    int64_t ctiles, qtiles, ctiles_per_xcd;   // filled by launch_filter
};

int64_t mfma_kp(int P);
sfc_status launch_dict_operand(const uint8_t* xq, const uint32_t* dict, int64_t n,
                               const int32_t* elem_off, int P, int C, uint16_t* B, hipStream_t st);
sfc_status launch_query_operand(const float* t, const uint8_t* m, int64_t Q, int64_t Qpad, int Kd,
                                int C, const float* qp, uint16_t* A, int32_t* T2, int32_t* kq,
                                int32_t* flag, hipStream_t st);
sfc_status launch_filter(FilterArgs a, int pass, hipStream_t st);
sfc_status launch_threshold(const int32_t* eqmin, const int32_t* kq, const int32_t* flag,
                            const float* qp, int64_t Q, int32_t* thr, hipStream_t st);
// exact rescoring of each query's candidate list; fb[q] = 1 when the list
// overflowed or the threshold was invalid (the float32 scan must answer q)
sfc_status launch_list_rescore(const Grid& g, const float* vol, const float* t,
                               const uint32_t* rowmask, int64_t qpad, const uint32_t* list,
                               const int32_t* cnt, const int32_t* thr, int cap, int64_t Q,
                               int64_t* best_id, float* best_cost, uint8_t* fb, hipStream_t st);

}  // namespace sfc
