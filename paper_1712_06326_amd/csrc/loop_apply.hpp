// The fill loop's apply step as a device function, shared by the apply
// kernel and by the index query's split rescoring, whose last workgroup
// applies a lone target's answer without another launch.
#pragma once

#include "inpaint.hpp"

namespace sfc {

__device__ inline void coords_of(const Grid& g, int64_t v, int64_t* c) {
    for (int i = 0; i < g.nd; i++) {
        c[i] = v / g.stride[i];
        v -= c[i] * g.stride[i];
    }
}

// Applies the pending answer with one workgroup of any size: copies the
// patch at s (thread 0's s0; -1 for none) into the unknown in-bounds voxels
// of the target's box, marks them known with the target's confidence, logs
// the iteration (cost: thread 0's c0) and counts the filled voxels. With
// nothing pending it returns at once (every thread reads the same state).
__device__ inline void apply_pending(const LoopApply& a, int64_t s0, float c0) {
    __shared__ int64_t sh_s;
    __shared__ float sh_cost;
    __shared__ int sh_filled;
    LoopState* ls = a.ls;
    const Grid& g = a.g;
    // nothing pending: the last fill (applied by a standalone apply at the
    // start of a round) keeps its region marked for the update that follows
    if (!ls->pending) return;
    const int64_t p = ls->centre;
    if (threadIdx.x == 0) {
        sh_s = s0;
        sh_cost = c0;
        sh_filled = 0;
    }
    __syncthreads();
    const int64_t s = sh_s;
    if (s >= 0) {
        int64_t cp[kMaxDims], cs[kMaxDims];
        coords_of(g, p, cp);
        coords_of(g, s, cs);
        const double cpick = ls->cpick;
        // r / K as a multiply-high: exact while r * K < 2^32 (r < K^d <= 2197)
        const uint32_t kinv = 0xffffffffu / (uint32_t)g.K + 1u;
        int filled = 0;
        for (int rho = threadIdx.x; rho < g.Kd; rho += blockDim.x) {
            int64_t up = 0, us = 0;
            bool inb = true;
            uint32_t r = (uint32_t)rho;
            for (int ax = g.nd - 1; ax >= 0; ax--) {
                const uint32_t rq = __umulhi(r, kinv);
                const int64_t o = (int64_t)(r - rq * (uint32_t)g.K) - g.h;
                r = rq;
                const int64_t x = cp[ax] + o;
                if (x < 0 || x >= g.shape[ax]) inb = false;
                up += x * g.stride[ax];
                us += (cs[ax] + o) * g.stride[ax];
            }
            // the target voxel's mask and the source values requested
            // together: the source patch lies inside the volume and is all
            // known, so it never overlaps the voxels written here
            const uint8_t known = a.mask[inb ? up : p];
            float sv[kMaxChannels];
#pragma unroll
            for (int ch = 0; ch < kMaxChannels; ch++)
                if (ch < g.C) sv[ch] = a.vol[us * g.C + ch];
            if (!inb || known) continue;
#pragma unroll
            for (int ch = 0; ch < kMaxChannels; ch++)
                if (ch < g.C) a.vol[up * g.C + ch] = sv[ch];
            a.mask[up] = 1;
            a.conf[up] = cpick;
            filled++;
        }
        if (filled) atomicAdd(&sh_filled, filled);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ls->pending = 0;
        if (s >= 0) {
            const int64_t it = ls->it;
            if (it < a.cap) {
                a.lc[it] = p;
                a.lsrc[it] = s;
                a.lcost[it] = sh_cost;
            }
            ls->it = it + 1;
            ls->last = p;
            ls->unknown -= (unsigned long long)sh_filled;
        } else {
            ls->last = -1;
        }
    }
}

}  // namespace sfc
