// Fill loop kernels (Section I: repeatedly pick a target on the fill front,
// find its best dictionary patch, insert it). The fill order follows
// Criminisi et al.'s priority, which the paper cites without formulas; the
// formulas below are the documented reading: P = C_p * D_p with
//   C_p = (sum of confidence over the known in-bounds voxels of the box, rho
//         ascending) / K^nd,
//   D_p = |grad I^perp . n| (2D) or |grad I x n| (3D), I = channel mean,
//         grad I by central differences where both neighbours are known,
//         one-sided where one is, else 0; n = the difference of the known
//         indicator across p (out of bounds counts as known), normalised.
// All arithmetic is float64 without fused operations, in the same order as
// the reference implementation, so the chosen targets agree bit for bit.
#include "loop_apply.hpp"

namespace sfc {

namespace {

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}


__device__ inline double mean_intensity(const float* vol, int64_t v, int C) {
    double s = 0.0;
    for (int ch = 0; ch < C; ch++) s += (double)vol[v * C + ch];
    return s / (double)C;
}

struct Cand {
    double p, c;
    int64_t id;
};

// a better than b: larger priority, then larger confidence, then lower id
__device__ inline bool better(const Cand& a, const Cand& b) {
    if (a.p != b.p) return a.p > b.p;
    if (a.c != b.c) return a.c > b.c;
    return a.id < b.id;
}

__device__ inline Cand shfl_cand(const Cand& x, int off) {
    Cand y;
    y.p = __shfl_xor(x.p, off, 64);
    y.c = __shfl_xor(x.c, off, 64);
    y.id = __shfl_xor(x.id, off, 64);
    return y;
}

// The candidate of front voxel v (coordinates c) whose box confidence sum
// is cs: (P, C, id) under order 0 (Criminisi), (-C, 0, id) under order 1
// (raster: only the id ranks, C is carried for the confidence update).
// What the data term reads around voxel v: its channel mean and, per
// axis, the two neighbours' mask bytes (0 outside) and channel means. All
// of them are requested at once: a mean is read whether or not its
// neighbour is known (an outside neighbour reads v itself) and dropped
// when unused, so the values and the arithmetic are those of the reading
// that branches first.
struct Nbrs {
    double I0, Ip[kMaxDims], Im[kMaxDims];
    uint8_t mp[kMaxDims], mm[kMaxDims];
};

__device__ inline Nbrs load_nbrs(const float* __restrict__ vol, const uint8_t* __restrict__ mask,
                                 const Grid& g, int64_t v, const int64_t* c) {
    Nbrs n;
    n.I0 = mean_intensity(vol, v, g.C);
#pragma unroll
    for (int i = 0; i < kMaxDims; i++) {   // static indices: the arrays stay in registers
        n.mp[i] = n.mm[i] = 0;
        n.Ip[i] = n.Im[i] = 0.0;
        if (i >= g.nd) continue;
        const bool hasp = c[i] + 1 < g.shape[i], hasm = c[i] > 0;
        const int64_t vp = hasp ? v + g.stride[i] : v, vm = hasm ? v - g.stride[i] : v;
        const uint8_t bp = mask[vp], bm = mask[vm];
        n.mp[i] = hasp ? bp : 0;
        n.mm[i] = hasm ? bm : 0;
        n.Ip[i] = mean_intensity(vol, vp, g.C);
        n.Im[i] = mean_intensity(vol, vm, g.C);
    }
    return n;
}

__device__ inline Cand cand_from_nbrs(const Nbrs& n, const Grid& g, int order, int64_t v,
                                      const int64_t* c, double cs) {
    const double Cp = cs / (double)g.Kd;
    if (order != 0) return Cand{-Cp, 0.0, v};   // carried, not compared (see reduce with order 1)
    double gr[kMaxDims], nr[kMaxDims], nn = 0.0;
    const double I0 = n.I0;
#pragma unroll
    for (int i = 0; i < kMaxDims; i++) {
        gr[i] = nr[i] = 0.0;
        if (i >= g.nd) continue;
        const bool hasp = c[i] + 1 < g.shape[i], hasm = c[i] > 0;
        const bool kp = n.mp[i] != 0, km = n.mm[i] != 0;
        if (kp && km)
            gr[i] = (n.Ip[i] - n.Im[i]) / 2.0;
        else if (kp)
            gr[i] = n.Ip[i] - I0;
        else if (km)
            gr[i] = I0 - n.Im[i];
        else
            gr[i] = 0.0;
        const int ip = hasp ? n.mp[i] : 1, im = hasm ? n.mm[i] : 1;
        nr[i] = (double)(ip - im);
        nn += nr[i] * nr[i];
    }
    double Dp = 0.0;
    if (nn > 0.0) {
        const double len = sqrt(nn);
#pragma unroll
        for (int i = 0; i < kMaxDims; i++)
            if (i < g.nd) nr[i] = nr[i] / len;
        if (g.nd == 2) {
            Dp = fabs(gr[0] * nr[1] - gr[1] * nr[0]);
        } else {
            const double c0 = gr[1] * nr[2] - gr[2] * nr[1];
            const double c1 = gr[2] * nr[0] - gr[0] * nr[2];
            const double c2 = gr[0] * nr[1] - gr[1] * nr[0];
            Dp = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        }
    }
    return Cand{Cp * Dp, Cp, v};
}

__device__ inline Cand cand_from_box(const float* __restrict__ vol, const uint8_t* __restrict__ mask,
                                     const Grid& g, int order, int64_t v, const int64_t* c,
                                     double cs) {
    if (order != 0) return Cand{-(cs / (double)g.Kd), 0.0, v};
    return cand_from_nbrs(load_nbrs(vol, mask, g, v, c), g, order, v, c, cs);
}

// The fill-order candidate of voxel v: cand_from_box for a front voxel,
// {-1, -1, max} otherwise.
__device__ inline Cand voxel_cand(const float* __restrict__ vol, const uint8_t* __restrict__ mask,
                                  const double* __restrict__ conf, const Grid& g, int order,
                                  int64_t v) {
    if (!mask[v]) return Cand{-1.0, -1.0, INT64_MAX};
    int64_t c[kMaxDims];
    coords_of(g, v, c);
    bool front = false;
    for (int i = 0; i < g.nd; i++) {
        if (c[i] > 0 && !mask[v - g.stride[i]]) front = true;
        if (c[i] + 1 < g.shape[i] && !mask[v + g.stride[i]]) front = true;
    }
    if (!front) return Cand{-1.0, -1.0, INT64_MAX};
    double cs = 0.0;
    for (int rho = 0; rho < g.Kd; rho++) {
        int64_t u = 0;
        bool inb = true;
        int r = rho;
        for (int a = g.nd - 1; a >= 0; a--) {
            const int64_t x = c[a] + (r % g.K) - g.h;
            r /= g.K;
            if (x < 0 || x >= g.shape[a]) inb = false;
            u += x * g.stride[a];
        }
        if (inb && mask[u]) cs += conf[u];
    }
    return cand_from_box(vol, mask, g, order, v, c, cs);
}

__device__ inline bool ranks_before(const Cand& a, const Cand& b, int order) {
    return order == 0 ? better(a, b) : (a.id < b.id);
}

// Per block: the best front voxel by (P, C, -id) (order 0) or the lowest
// front id (order 1, with P and C of that voxel), and the unknown count.
__global__ __launch_bounds__(256) void priority_kernel(const float* __restrict__ vol,
                                                       const uint8_t* __restrict__ mask,
                                                       const double* __restrict__ conf, Grid g,
                                                       int order, Cand* __restrict__ part,
                                                       unsigned long long* __restrict__ unknown) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Cand best{-1.0, -1.0, INT64_MAX};
    int unk = 0;
    if (v < g.nvox) {
        if (!mask[v]) unk = 1;
        else best = voxel_cand(vol, mask, conf, g, order, v);
    }
    // block reduction
    for (int off = 32; off > 0; off >>= 1) {
        const Cand o = shfl_cand(best, off);
        if (order == 0 ? better(o, best) : (o.id < best.id)) best = o;
        unk += __shfl_xor(unk, off, 64);
    }
    __shared__ Cand sb[4];
    __shared__ int su[4];
    if ((threadIdx.x & 63) == 0) {
        sb[threadIdx.x >> 6] = best;
        su[threadIdx.x >> 6] = unk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Cand b = sb[0];
        int u = su[0];
        for (int w = 1; w < 4; w++) {
            if (order == 0 ? better(sb[w], b) : (sb[w].id < b.id)) b = sb[w];
            u += su[w];
        }
        part[blockIdx.x] = b;
        if (u) atomicAdd(unknown, (unsigned long long)u);
    }
}

__global__ __launch_bounds__(256) void pick_kernel(const Cand* __restrict__ part, int64_t nb, int order,
                                                   int64_t* __restrict__ centre, double* __restrict__ cpick) {
    Cand best{-1.0, -1.0, INT64_MAX};
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
        const Cand o = part[i];
        if (order == 0 ? better(o, best) : (o.id < best.id)) best = o;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const Cand o = shfl_cand(best, off);
        if (order == 0 ? better(o, best) : (o.id < best.id)) best = o;
    }
    __shared__ Cand sb[4];
    if ((threadIdx.x & 63) == 0) sb[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        Cand b = sb[0];
        for (int w = 1; w < 4; w++)
            if (order == 0 ? better(sb[w], b) : (sb[w].id < b.id)) b = sb[w];
        *centre = b.id == INT64_MAX ? -1 : b.id;
        *cpick = order == 0 ? b.c : -b.p;
    }
}

// Copy the chosen patch into the unknown in-bounds voxels of the target box,
// mark them known and give them the target's confidence; log the iteration.
__global__ void fill_kernel(float* __restrict__ vol, uint8_t* __restrict__ mask,
                            double* __restrict__ conf, Grid g, const int64_t* __restrict__ centre,
                            const int64_t* __restrict__ source, const float* __restrict__ cost,
                            const double* __restrict__ cpick, int64_t it, int64_t cap,
                            int64_t* __restrict__ lc, int64_t* __restrict__ ls,
                            float* __restrict__ lcost) {
    const int rho = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = *centre, s = *source;
    if (rho == 0 && it < cap) {
        lc[it] = p;
        ls[it] = s;
        lcost[it] = *cost;
    }
    if (rho >= g.Kd || p < 0 || s < 0) return;
    int64_t cp[kMaxDims], cs[kMaxDims];
    coords_of(g, p, cp);
    coords_of(g, s, cs);
    int64_t up = 0, us = 0;
    bool inb = true;
    int r = rho;
    for (int a = g.nd - 1; a >= 0; a--) {
        const int64_t o = (r % g.K) - g.h;
        r /= g.K;
        const int64_t x = cp[a] + o;
        if (x < 0 || x >= g.shape[a]) inb = false;
        up += x * g.stride[a];
        us += (cs[a] + o) * g.stride[a];
    }
    if (!inb || mask[up]) return;
    for (int ch = 0; ch < g.C; ch++) vol[up * g.C + ch] = vol[us * g.C + ch];
    mask[up] = 1;
    conf[up] = *cpick;
}

// ---- the device-resident loop: priorities kept per voxel and updated only
// around the last filled box, block partials in two levels, loop state on
// the device.

// Best candidate of a 256-thread block (x valid in every thread).
__device__ inline Cand block_best(Cand x, int order) {
    for (int off = 32; off > 0; off >>= 1) {
        const Cand o = shfl_cand(x, off);
        if (ranks_before(o, x, order)) x = o;
    }
    __shared__ Cand sb[4];
    if ((threadIdx.x & 63) == 0) sb[threadIdx.x >> 6] = x;
    __syncthreads();
    Cand b = sb[0];
    for (int w = 1; w < 4; w++)
        if (ranks_before(sb[w], b, order)) b = sb[w];
    return b;
}

__global__ __launch_bounds__(256) void cand_all_kernel(const float* __restrict__ vol,
                                                       const uint8_t* __restrict__ mask,
                                                       const double* __restrict__ conf, Grid g,
                                                       int order, Cand* __restrict__ pv) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < g.nvox) pv[v] = voxel_cand(vol, mask, conf, g, order, v);
}

// part[b] = best of src[256 b .. 256 b + 255] (src has n entries)
__global__ __launch_bounds__(256) void part_all_kernel(const Cand* __restrict__ src, int64_t n,
                                                       int order, Cand* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const Cand x = i < n ? src[i] : Cand{-1.0, -1.0, INT64_MAX};
    const Cand b = block_best(x, order);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ void count_unknown_kernel(const uint8_t* __restrict__ mask, int64_t n,
                                     LoopState* __restrict__ ls) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int u = (i < n && !mask[i]) ? 1 : 0;
    const unsigned long long b = __ballot(u);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&ls->unknown, (unsigned long long)__popcll(b));
}

__global__ void loop_init_kernel(LoopState* ls) {
    ls->unknown = 0;
    ls->centre = -1;
    ls->cpick = 0.0;
    ls->source = -1;
    ls->cost = 0.0f;
    ls->last = -1;
    ls->it = 0;
    ls->pending = 0;
}

// The region whose candidates a fill at centre p can change: the box of
// half-width K-1 around p (the confidence box sum of a voxel reaches h
// around it, the filled box h around p; front status and gradients reach one
// voxel around the filled box, and h + 1 <= K - 1 for K >= 3), clipped.
// Line l of the region: its coordinates along the slower axes, and the id
// range of its clipped extent along the fastest axis; false if the line is
// outside the volume.
__device__ inline bool region_line(const Grid& g, int64_t p, int64_t l, int64_t* id0, int64_t* id1) {
    const int R = g.K - 1, side = 2 * R + 1;
    int64_t c[kMaxDims];
    coords_of(g, p, c);
    int64_t base = 0;
    for (int a = g.nd - 2; a >= 0; a--) {
        const int64_t x = c[a] + (l % side) - R;
        l /= side;
        if (x < 0 || x >= g.shape[a]) return false;
        base += x * g.stride[a];
    }
    const int f = g.nd - 1;
    const int64_t x0 = c[f] - R < 0 ? 0 : c[f] - R;
    const int64_t x1 = c[f] + R >= g.shape[f] ? g.shape[f] - 1 : c[f] + R;
    *id0 = base + x0;
    *id1 = base + x1;
    return true;
}

__device__ inline int64_t region_lines(const Grid& g) {
    int64_t n = 1;
    for (int a = 0; a < g.nd - 1; a++) n *= 2 * g.K - 1;
    return n;
}

// candidates of the region around the last filled centre: one wave per
// voxel of the region, four per workgroup. The lanes load the voxel's box
// (confidence where known and in bounds, else +0, which leaves the sum
// unchanged) into LDS in parallel; lane 0 then adds them in ascending rho,
// the definition's order, and finishes the candidate.
constexpr int kBoxChunk = 512;   // box values staged per wave at a time
__global__ __launch_bounds__(256) void region_cand_kernel(const float* __restrict__ vol,
                                                          const uint8_t* __restrict__ mask,
                                                          const double* __restrict__ conf, Grid g,
                                                          int order, const LoopState* __restrict__ ls,
                                                          Cand* __restrict__ pv) {
    __shared__ double box_lds[4][kBoxChunk];
    const int64_t p = ls->last;
    if (p < 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int R = g.K - 1, side = 2 * R + 1;
    int64_t nreg = 1;
    for (int a = 0; a < g.nd; a++) nreg *= side;
    const int64_t k = (int64_t)blockIdx.x * 4 + wave;
    if (k >= nreg) return;
    // the region voxel: offsets in [-R, R] per axis, last axis fastest
    int64_t cp[kMaxDims], c[kMaxDims];
    coords_of(g, p, cp);
    int64_t kk = k, v = 0;
    for (int a = g.nd - 1; a >= 0; a--) {
        c[a] = cp[a] + (kk % side) - R;
        kk /= side;
        if (c[a] < 0 || c[a] >= g.shape[a]) return;
        v += c[a] * g.stride[a];
    }
    // the voxel's mask and its face neighbours' requested together (an
    // outside neighbour reads the voxel itself and is not used)
    const uint8_t mv = mask[v];
    uint8_t mlo[kMaxDims], mhi[kMaxDims];
#pragma unroll
    for (int i = 0; i < kMaxDims; i++) {
        mlo[i] = mhi[i] = 1;
        if (i >= g.nd) continue;
        mlo[i] = mask[c[i] > 0 ? v - g.stride[i] : v];
        mhi[i] = mask[c[i] + 1 < g.shape[i] ? v + g.stride[i] : v];
    }
    if (!mv) {
        if (lane == 0) pv[v] = Cand{-1.0, -1.0, INT64_MAX};
        return;
    }
    bool front = false;
#pragma unroll
    for (int i = 0; i < kMaxDims; i++) {
        if (i >= g.nd) continue;
        if (c[i] > 0 && !mlo[i]) front = true;
        if (c[i] + 1 < g.shape[i] && !mhi[i]) front = true;
    }
    if (!front) {
        if (lane == 0) pv[v] = Cand{-1.0, -1.0, INT64_MAX};
        return;
    }
    // the data term's neighbour values, requested with the box's loads
    Nbrs nb;
    if (lane == 0 && order == 0) nb = load_nbrs(vol, mask, g, v, c);
    double* bx = box_lds[wave];
    double cs = 0.0;
    // r / K as a multiply-high: exact while r * K < 2^32 (r < K^d <= 2197)
    const uint32_t kinv = 0xffffffffu / (uint32_t)g.K + 1u;
    for (int base = 0; base < g.Kd; base += kBoxChunk) {
        const int n = g.Kd - base < kBoxChunk ? g.Kd - base : kBoxChunk;
#pragma unroll 4
        for (int i = lane; i < n; i += 64) {
            int64_t u = 0;
            bool inb = true;
            uint32_t r = (uint32_t)(base + i);
            for (int a = g.nd - 1; a >= 0; a--) {
                const uint32_t rq = __umulhi(r, kinv);
                const int64_t x = c[a] + (int64_t)(r - rq * (uint32_t)g.K) - g.h;
                r = rq;
                if (x < 0 || x >= g.shape[a]) inb = false;
                u += x * g.stride[a];
            }
            // mask and confidence requested together (an outside offset
            // reads the voxel itself, then is dropped)
            const int64_t uu = inb ? u : v;
            const uint8_t mk = mask[uu];
            const double cf = conf[uu];
            bx[i] = (inb && mk) ? cf : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the oracle's order, one add after another; the LDS reads go out
        // 32 at a time ahead of their adds
        if (lane == 0) {
            int i = 0;
            for (; i + 32 <= n; i += 32) {
                double x[32];
#pragma unroll
                for (int k = 0; k < 32; k++) x[k] = bx[i + k];
#pragma unroll
                for (int k = 0; k < 32; k++) cs += x[k];
            }
            for (; i < n; i++) cs += bx[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane == 0) pv[v] = cand_from_nbrs(nb, g, order, v, c, cs);
}

__device__ inline Cand wave_best(Cand x, int order) {
    for (int off = 32; off > 0; off >>= 1) {
        const Cand o = shfl_cand(x, off);
        if (ranks_before(o, x, order)) x = o;
    }
    return x;
}

// Applies the previous iteration's answer (pending), apply_pending with
// one workgroup. best: the float32 scan's packed (cost bits << 32 | id), or
// null when the query wrote source and cost into the state.
__global__ __launch_bounds__(256) void loop_apply_kernel(LoopApply a,
                                                         const uint64_t* __restrict__ best) {
    int64_t s0 = -1;
    float c0 = 0.0f;
    if (threadIdx.x == 0) {
        s0 = a.ls->source;
        c0 = a.ls->cost;
        if (best) {
            const uint64_t b = best[0];
            s0 = b == ~0ull ? -1 : (int64_t)(b & 0xffffffffull);
            c0 = __uint_as_float((uint32_t)(b >> 32));
        }
    }
    apply_pending(a, s0, c0);
}

// level-1 partials of the blocks of 256 voxels that the last fill's region
// touches: a workgroup per (region line, block); lines that share a block
// write the same value
__global__ __launch_bounds__(256) void loop_part1_kernel(const Cand* __restrict__ pv, Grid g,
                                                         int order, const LoopState* __restrict__ ls,
                                                         Cand* __restrict__ part1) {
    const int64_t p = ls->last;
    if (p < 0) return;
    int64_t id0, id1;
    if (!region_line(g, p, blockIdx.x >> 1, &id0, &id1)) return;
    const int64_t b = id0 / 256 + (blockIdx.x & 1);
    if (b > id1 / 256) return;
    const int64_t i = b * 256 + threadIdx.x;
    const Cand x = i < g.nvox ? pv[i] : Cand{-1.0, -1.0, INT64_MAX};
    const Cand best = block_best(x, order);
    if (threadIdx.x == 0) part1[b] = best;
}

// level-2 partials over the level-1 blocks that changed
__global__ __launch_bounds__(256) void loop_part2_kernel(const Cand* __restrict__ part1,
                                                         int64_t nb1, Grid g, int order,
                                                         const LoopState* __restrict__ ls,
                                                         Cand* __restrict__ part2) {
    const int64_t p = ls->last;
    if (p < 0) return;
    int64_t id0, id1;
    if (!region_line(g, p, blockIdx.x >> 1, &id0, &id1)) return;
    const int64_t b = id0 / 256 + (blockIdx.x & 1);
    if (b > id1 / 256) return;
    const int64_t c = b / 256;
    const int64_t i = c * 256 + threadIdx.x;
    const Cand x = i < nb1 ? part1[i] : Cand{-1.0, -1.0, INT64_MAX};
    const Cand best = block_best(x, order);
    if (threadIdx.x == 0) part2[c] = best;
}

// One workgroup: the next target from the top partial level, and its
// extraction (t, m; for the float32 scan also query slot 0 of the padded
// targets and row masks, and a cleared result).
constexpr int kSelThreads = 1024;
constexpr int64_t kOneLevel = 16384;   // level-1 entries the pick reads directly (4M voxels)
__global__ __launch_bounds__(kSelThreads) void loop_select_kernel(
    const float* __restrict__ vol, const uint8_t* __restrict__ mask, Grid g, int order,
    const Cand* __restrict__ pv, Cand* __restrict__ part1, int64_t nb1, Cand* __restrict__ part2,
    int64_t nb2, LoopState* __restrict__ ls, float* __restrict__ t, uint8_t* __restrict__ m,
    float* __restrict__ tp, uint32_t* __restrict__ rm, int64_t qpad, uint64_t* __restrict__ best) {
    constexpr int NW = kSelThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Cand none{-1.0, -1.0, INT64_MAX};
    // the next target
    __shared__ Cand sb[NW];
    __shared__ int64_t sh_centre;
    Cand x = none;
    const Cand* top = nb1 > kOneLevel ? part2 : part1;
    const int64_t ntop = nb1 > kOneLevel ? nb2 : nb1;
    for (int64_t i = threadIdx.x; i < ntop; i += kSelThreads)
        if (ranks_before(top[i], x, order)) x = top[i];
    x = wave_best(x, order);
    if (lane == 0) sb[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        Cand b = sb[0];
        for (int w = 1; w < NW; w++)
            if (ranks_before(sb[w], b, order)) b = sb[w];
        const bool nothing = b.id == INT64_MAX || ls->unknown == 0;
        const int64_t c = nothing ? -1 : b.id;
        ls->centre = c;
        ls->cpick = order == 0 ? b.c : -b.p;
        ls->pending = c >= 0 ? 1 : 0;
        sh_centre = c;
        if (best) best[0] = ~0ull;
    }
    __syncthreads();
    const int64_t c = sh_centre;
    if (c < 0) return;
    // extraction of the target at c
    int64_t cc[kMaxDims];
    coords_of(g, c, cc);
    // r / K as a multiply-high: exact while r * K < 2^32 (r < K^d <= 2197)
    const uint32_t kinv = 0xffffffffu / (uint32_t)g.K + 1u;
    for (int rho = threadIdx.x; rho < g.Kd; rho += kSelThreads) {
        int64_t v = 0;
        bool inb = true;
        uint32_t r = (uint32_t)rho;
        for (int a = g.nd - 1; a >= 0; a--) {
            const uint32_t rq = __umulhi(r, kinv);
            const int64_t xx = cc[a] + (int64_t)(r - rq * (uint32_t)g.K) - g.h;
            r = rq;
            if (xx < 0 || xx >= g.shape[a]) inb = false;
            v += xx * g.stride[a];
        }
        // mask and values requested together (an outside offset reads the
        // centre, then is dropped)
        const int64_t vv = inb ? v : c;
        const bool known = inb && mask[vv];
        m[rho] = known ? 1 : 0;
        for (int ch = 0; ch < g.C; ch++) {
            const float x = vol[vv * g.C + ch];
            const float val = known ? x : 0.0f;
            t[rho * g.C + ch] = val;
            if (tp) tp[rho * g.C + ch] = val;
        }
    }
    if (rm) {
        // row r of the patch: bit dx set when pixel r*K + dx is known
        for (int r = threadIdx.x; r < g.rows; r += kSelThreads) {
            int rr = r;
            int64_t base = 0;
            bool inrow = true;
            for (int a = g.nd - 2; a >= 0; a--) {
                const int64_t xx = cc[a] + (rr % g.K) - g.h;
                rr /= g.K;
                if (xx < 0 || xx >= g.shape[a]) inrow = false;
                base += xx * g.stride[a];
            }
            uint32_t bits = 0;
            const int f = g.nd - 1;
            for (int dx = 0; dx < g.K; dx++) {
                const int64_t xx = cc[f] + dx - g.h;
                const bool in = inrow && xx >= 0 && xx < g.shape[f];
                const uint8_t mk = mask[in ? base + xx : c];   // loads not behind a branch
                if (in && mk) bits |= 1u << dx;
            }
            rm[(int64_t)r * qpad] = bits;
        }
    }
}

__global__ void conf_init_kernel(const uint8_t* __restrict__ mask, int64_t n, double* __restrict__ conf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) conf[i] = mask[i] ? 1.0 : 0.0;
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

}  // namespace

size_t inpaint_part_bytes(const Grid& g) { return (size_t)blocks_for(g.nvox) * sizeof(Cand); }

sfc_status launch_conf_init(const uint8_t* mask, const Grid& g, double* conf, hipStream_t st) {
    conf_init_kernel<<<blocks_for(g.nvox), 256, 0, st>>>(mask, g.nvox, conf);
    return launched("conf_init_kernel");
}

sfc_status launch_pick(const float* vol, const uint8_t* mask, const double* conf, const Grid& g,
                       int order, void* part, unsigned long long* unknown, int64_t* centre,
                       double* cpick, hipStream_t st) {
    zero_u64_kernel<<<1, 1, 0, st>>>(unknown);
    SFC_TRY(launched("zero_u64_kernel"));
    const unsigned nb = blocks_for(g.nvox);
    priority_kernel<<<nb, 256, 0, st>>>(vol, mask, conf, g, order, static_cast<Cand*>(part), unknown);
    SFC_TRY(launched("priority_kernel"));
    pick_kernel<<<1, 256, 0, st>>>(static_cast<const Cand*>(part), nb, order, centre, cpick);
    return launched("pick_kernel");
}

size_t loop_part_entries(const Grid& g, int64_t* nb1, int64_t* nb2) {
    *nb1 = (g.nvox + 255) / 256;
    *nb2 = (*nb1 + 255) / 256;
    return (size_t)(*nb1 + *nb2);
}
size_t loop_cand_bytes() { return sizeof(Cand); }

sfc_status launch_loop_init(const float* vol, const uint8_t* mask, const double* conf, const Grid& g,
                            int order, void* pv, void* part1, void* part2, LoopState* ls,
                            hipStream_t st) {
    int64_t nb1, nb2;
    loop_part_entries(g, &nb1, &nb2);
    loop_init_kernel<<<1, 1, 0, st>>>(ls);
    SFC_TRY(launched("loop_init_kernel"));
    count_unknown_kernel<<<blocks_for(g.nvox), 256, 0, st>>>(mask, g.nvox, ls);
    SFC_TRY(launched("count_unknown_kernel"));
    cand_all_kernel<<<blocks_for(g.nvox), 256, 0, st>>>(vol, mask, conf, g, order, static_cast<Cand*>(pv));
    SFC_TRY(launched("cand_all_kernel"));
    part_all_kernel<<<(unsigned)nb1, 256, 0, st>>>(static_cast<const Cand*>(pv), g.nvox, order,
                                                   static_cast<Cand*>(part1));
    SFC_TRY(launched("part_all_kernel"));
    part_all_kernel<<<(unsigned)nb2, 256, 0, st>>>(static_cast<const Cand*>(part1), nb1, order,
                                                   static_cast<Cand*>(part2));
    return launched("part_all_kernel");
}

sfc_status launch_loop_apply(float* vol, uint8_t* mask, double* conf, const Grid& g, LoopState* ls,
                             const uint64_t* best, int64_t cap, int64_t* lc, int64_t* lsrc,
                             float* lcost, hipStream_t st) {
    const LoopApply a{vol, mask, conf, g, ls, cap, lc, lsrc, lcost};
    loop_apply_kernel<<<1, 256, 0, st>>>(a, best);
    return launched("loop_apply_kernel");
}

sfc_status launch_loop_select(const float* vol, const uint8_t* mask, const double* conf,
                              const Grid& g, int order, void* pv, void* part1, void* part2,
                              LoopState* ls, float* t, uint8_t* m, float* tp, uint32_t* rm,
                              int64_t qpad, uint64_t* best, hipStream_t st) {
    int64_t nb1, nb2;
    loop_part_entries(g, &nb1, &nb2);
    int64_t nreg = 1;
    for (int a = 0; a < g.nd; a++) nreg *= 2 * g.K - 1;
    region_cand_kernel<<<(unsigned)((nreg + 3) / 4), 256, 0, st>>>(vol, mask, conf, g, order, ls,
                                                                 static_cast<Cand*>(pv));
    SFC_TRY(launched("region_cand_kernel"));
    int64_t lines = 1;
    for (int a = 0; a < g.nd - 1; a++) lines *= 2 * g.K - 1;
    loop_part1_kernel<<<(unsigned)(2 * lines), 256, 0, st>>>(static_cast<const Cand*>(pv), g, order,
                                                             ls, static_cast<Cand*>(part1));
    SFC_TRY(launched("loop_part1_kernel"));
    if (nb1 > kOneLevel) {
        loop_part2_kernel<<<(unsigned)(2 * lines), 256, 0, st>>>(static_cast<const Cand*>(part1), nb1,
                                                                 g, order, ls,
                                                                 static_cast<Cand*>(part2));
        SFC_TRY(launched("loop_part2_kernel"));
    }
    loop_select_kernel<<<1, kSelThreads, 0, st>>>(vol, mask, g, order, static_cast<const Cand*>(pv),
                                                  static_cast<Cand*>(part1), nb1,
                                                  static_cast<Cand*>(part2), nb2, ls, t, m, tp, rm,
                                                  qpad, best);
    return launched("loop_select_kernel");
}

sfc_status launch_fill(float* vol, uint8_t* mask, double* conf, const Grid& g, const int64_t* centre,
                       const int64_t* source, const float* cost, const double* cpick, int64_t it,
                       int64_t cap, int64_t* lc, int64_t* ls, float* lcost, hipStream_t st) {
    fill_kernel<<<blocks_for(g.Kd), 256, 0, st>>>(vol, mask, conf, g, centre, source, cost, cpick, it,
                                                  cap, lc, ls, lcost);
    return launched("fill_kernel");
}

}  // namespace sfc
