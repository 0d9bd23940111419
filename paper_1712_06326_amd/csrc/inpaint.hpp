// Fill loop kernels.
#pragma once

#include "common.hpp"

namespace sfc {

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
