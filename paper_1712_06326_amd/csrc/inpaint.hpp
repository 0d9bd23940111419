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
    int64_t last;                 // centre filled by the previous iteration (-1: none)
    int64_t it;                   // iterations done
};

// entries of the two partial levels (nb1 = blocks of 256 voxels, nb2 =
// blocks of 256 level-1 entries); bytes of one entry
size_t loop_part_entries(const Grid& g, int64_t* nb1, int64_t* nb2);
size_t loop_cand_bytes();
// loop state, unknown count, every voxel's candidate and both partial levels
sfc_status launch_loop_init(const float* vol, const uint8_t* mask, const double* conf, const Grid& g,
                            int order, void* pv, void* part1, void* part2, LoopState* ls,
                            hipStream_t st);
// candidates and partials around the last filled centre, then the next target
sfc_status launch_loop_pick(const float* vol, const uint8_t* mask, const double* conf, const Grid& g,
                            int order, void* pv, void* part1, void* part2, LoopState* ls,
                            hipStream_t st);
// copy the chosen patch, log the iteration, count it
sfc_status launch_loop_fill(float* vol, uint8_t* mask, double* conf, const Grid& g, LoopState* ls,
                            int64_t cap, int64_t* lc, int64_t* lsrc, float* lcost, hipStream_t st);

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
