// Fill loop kernels.
#pragma once

#include "common.hpp"

namespace sfc {

// State of the device-resident fill loop (device memory).
struct LoopState {
    unsigned long long unknown;   // unknown voxels left
    int64_t centre;               // this iteration's target (-1: none)
    double cpick;                 // its confidence
    int64_t source;               // its best patch
    float cost;
    float pad;
    int64_t last;                 // centre filled by the last apply (-1: none)
    int64_t it;                   // iterations done
    int32_t pending;              // 1: centre's query answer not applied yet
    int32_t pad2;
};

// What the loop's apply step writes: the volume, the known mask and
// confidences, the loop state and the iteration log (cap entries).
struct LoopApply {
    float* vol;
    uint8_t* mask;
    double* conf;
    Grid g;
    LoopState* ls;
    int64_t cap;
    int64_t* lc;
    int64_t* lsrc;
    float* lcost;
};

// entries of the two partial levels (nb1 = blocks of 256 voxels, nb2 =
// blocks of 256 level-1 entries); bytes of one entry
size_t loop_part_entries(const Grid& g, int64_t* nb1, int64_t* nb2);
size_t loop_cand_bytes();
// loop state, unknown count, every voxel's candidate and both partial levels
sfc_status launch_loop_init(const float* vol, const uint8_t* mask, const double* conf, const Grid& g,
                            int order, void* pv, void* part1, void* part2, LoopState* ls,
                            hipStream_t st);
// applies the pending answer (best: the float32 scan's packed result, or
// null when the query wrote source and cost into the state)
sfc_status launch_loop_apply(float* vol, uint8_t* mask, double* conf, const Grid& g, LoopState* ls,
                             const uint64_t* best, int64_t cap, int64_t* lc, int64_t* lsrc,
                             float* lcost, hipStream_t st);
// candidates and partials around the last fill, the next target and its
// extraction (t, m; with tp/rm/best non-null also the float32 scan's query
// slot 0 and a cleared result)
sfc_status launch_loop_select(const float* vol, const uint8_t* mask, const double* conf,
                              const Grid& g, int order, void* pv, void* part1, void* part2,
                              LoopState* ls, float* t, uint8_t* m, float* tp, uint32_t* rm,
                              int64_t qpad, uint64_t* best, hipStream_t st);

size_t inpaint_part_bytes(const Grid& g);
sfc_status launch_conf_init(const uint8_t* mask, const Grid& g, double* conf, hipStream_t st);
// chooses the next target: centre (-1 if the front is empty), its confidence,
// and the number of unknown voxels
sfc_status launch_pick(const float* vol, const uint8_t* mask, const double* conf, const Grid& g,
                       int order, void* part, unsigned long long* unknown, int64_t* centre,
                       double* cpick, hipStream_t st);
sfc_status launch_fill(float* vol, uint8_t* mask, double* conf, const Grid& g, const int64_t* centre,
                       const int64_t* source, const float* cost, const double* cpick, int64_t it,
                       int64_t cap, int64_t* lc, int64_t* ls, float* lcost, hipStream_t st);

}  // namespace sfc
