// Fill front, target extraction, dictionary validity and stream compaction.
#include "common.hpp"

namespace sfc {

namespace {

constexpr int kBlock = 256;
constexpr int kItemsPerThread = 16;
constexpr int kTile = kBlock * kItemsPerThread;

__device__ inline void coords_of(const Grid& g, int64_t v, int64_t* c) {
    for (int i = 0; i < g.nd; i++) {
        c[i] = v / g.stride[i];
        v -= c[i] * g.stride[i];
    }
}

// Known voxels with an unknown face neighbour (Fig. 1a).
__global__ void front_flags_kernel(const uint8_t* __restrict__ mask, Grid g,
                                   uint8_t* __restrict__ flags) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.nvox) return;
    uint8_t f = 0;
    if (mask[v]) {
        int64_t c[kMaxDims];
        coords_of(g, v, c);
        for (int i = 0; i < g.nd; i++) {
            if (c[i] > 0 && !mask[v - g.stride[i]]) f = 1;
            if (c[i] + 1 < g.shape[i] && !mask[v + g.stride[i]]) f = 1;
        }
    }
    flags[v] = f;
}

// One thread per (query, pixel): value and known flag of each target pixel.
__global__ void extract_kernel(const float* __restrict__ vol, const uint8_t* __restrict__ mask,
                               Grid g, const int64_t* __restrict__ centres, int64_t Q,
                               float* __restrict__ t, uint8_t* __restrict__ m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q * g.Kd) return;
    int64_t q = i / g.Kd;
    int rho = (int)(i - q * g.Kd);
    if (centres[q] < 0) {   // no target (an empty fill front): an all-unknown patch
        m[i] = 0;
        for (int ch = 0; ch < g.C; ch++) t[i * g.C + ch] = 0.0f;
        return;
    }
    int64_t c[kMaxDims];
    coords_of(g, centres[q], c);
    int64_t v = 0;
    bool inb = true;
    int r = rho;
    for (int a = g.nd - 1; a >= 0; a--) {
        int64_t x = c[a] + (r % g.K) - g.h;
        r /= g.K;
        if (x < 0 || x >= g.shape[a]) inb = false;
        v += x * g.stride[a];
    }
    bool known = inb && mask[v];
    m[i] = known ? 1 : 0;
    for (int ch = 0; ch < g.C; ch++) t[i * g.C + ch] = known ? vol[v * g.C + ch] : 0.0f;
}

// One axis of the box erosion: out[v] = 1 iff in[v + k*stride] for every
// k in [-h, h], all in bounds.
__global__ void erode_axis_kernel(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                  Grid g, int axis) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.nvox) return;
    int64_t c = (v / g.stride[axis]) % g.shape[axis];
    uint8_t ok = (c >= g.h && c < g.shape[axis] - g.h) ? 1 : 0;
    for (int k = -g.h; ok && k <= g.h; k++) ok = in[v + k * g.stride[axis]] ? 1 : 0;
    out[v] = ok;
}

__device__ inline int wave_incl_scan(int x) {
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive block scan of one int per thread (256 threads); returns the
// block total in *total.
__device__ inline int block_excl_scan(int x, int* total) {
    __shared__ int wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = wave_incl_scan(x);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int i = 0; i < kBlock / 64; i++) {
        if (i < w) pre += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - x;
}

__global__ void count_kernel(const uint8_t* __restrict__ flags, int64_t n,
                             int64_t* __restrict__ counts) {
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItemsPerThread;
    int c = 0;
    for (int k = 0; k < kItemsPerThread; k++) {
        int64_t i = base + k;
        if (i < n && flags[i]) c++;
    }
    int total;
    block_excl_scan(c, &total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Single-block exclusive scan over nb block counts; total -> *count_dev.
__global__ void scan_counts_kernel(int64_t* __restrict__ counts, int64_t nb,
                                   int64_t* __restrict__ count_dev) {
    __shared__ int64_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += kBlock) {
        int64_t i = base + threadIdx.x;
        int64_t x = (i < nb) ? counts[i] : 0;
        // 64-bit scan in two 32-bit halves is unnecessary: counts <= kTile
        int total;
        int pre = block_excl_scan((int)x, &total);
        int64_t carry = carry_s;
        if (i < nb) counts[i] = carry + pre;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count_dev = carry_s;
}

__global__ void scatter_kernel(const uint8_t* __restrict__ flags, int64_t n,
                               const int64_t* __restrict__ offsets, int64_t* __restrict__ out64,
                               uint32_t* __restrict__ out32, int64_t cap) {
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItemsPerThread;
    int c = 0;
    for (int k = 0; k < kItemsPerThread; k++) {
        int64_t i = base + k;
        if (i < n && flags[i]) c++;
    }
    int total;
    int pre = block_excl_scan(c, &total);
    int64_t pos = offsets[blockIdx.x] + pre;
    for (int k = 0; k < kItemsPerThread; k++) {
        int64_t i = base + k;
        if (i < n && flags[i]) {
            if (pos < cap) {
                if (out64) out64[pos] = i;
                else out32[pos] = (uint32_t)i;
            }
            pos++;
        }
    }
}

__global__ void fill_u64_kernel(uint64_t* p, int64_t n, uint64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void pad_f32_kernel(const float* __restrict__ in, int64_t n, int64_t npad,
                               float* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad) out[i] = i < n ? in[i] : 0.0f;
}

__global__ void u32_to_i64_kernel(const uint32_t* __restrict__ in, int64_t* __restrict__ out,
                                  int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

inline unsigned blocks_for(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

Grid make_grid(const sfc_geometry* gg, int K) {
    Grid g{};
    g.nd = gg->ndim;
    g.C = gg->channels;
    g.K = K;
    g.h = (K - 1) / 2;
    g.Kd = 1;
    for (int i = 0; i < g.nd; i++) g.Kd *= K;
    g.rows = g.Kd / K;
    g.nvox = 1;
    for (int i = g.nd - 1; i >= 0; i--) {
        g.shape[i] = gg->shape[i];
        g.stride[i] = g.nvox;
        g.nvox *= gg->shape[i];
    }
    return g;
}

static sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return check_hip(e, what);
    return SFC_OK;
}

sfc_status launch_front_flags(const uint8_t* mask, const Grid& g, uint8_t* flags, hipStream_t st) {
    if (g.nvox == 0) return SFC_OK;
    front_flags_kernel<<<blocks_for(g.nvox), kBlock, 0, st>>>(mask, g, flags);
    return launched("front_flags_kernel");
}

size_t compact_scratch_bytes(int64_t n) {
    int64_t nb = (n + kTile - 1) / kTile;
    return (size_t)(nb > 0 ? nb : 1) * sizeof(int64_t);
}

sfc_status launch_compact(const uint8_t* flags, int64_t n, int64_t* out64, uint32_t* out32,
                          int64_t cap, int64_t* count_dev, void* scratch, hipStream_t st) {
    int64_t nb = (n + kTile - 1) / kTile;
    int64_t* counts = static_cast<int64_t*>(scratch);
    if (nb > 0) {
        count_kernel<<<(unsigned)nb, kBlock, 0, st>>>(flags, n, counts);
        SFC_TRY(launched("count_kernel"));
    }
    scan_counts_kernel<<<1, kBlock, 0, st>>>(counts, nb, count_dev);
    SFC_TRY(launched("scan_counts_kernel"));
    if (nb > 0) {
        scatter_kernel<<<(unsigned)nb, kBlock, 0, st>>>(flags, n, counts, out64, out32, cap);
        SFC_TRY(launched("scatter_kernel"));
    }
    return SFC_OK;
}

sfc_status launch_extract(const float* vol, const uint8_t* mask, const Grid& g,
                          const int64_t* centres, int64_t Q, float* t, uint8_t* m,
                          hipStream_t st) {
    if (Q == 0) return SFC_OK;
    extract_kernel<<<blocks_for(Q * g.Kd), kBlock, 0, st>>>(vol, mask, g, centres, Q, t, m);
    return launched("extract_kernel");
}

sfc_status launch_valid_centres(const uint8_t* mask, const Grid& g, uint8_t* valid,
                                uint8_t* tmp, hipStream_t st) {
    unsigned nb = blocks_for(g.nvox);
    if (g.nd == 2) {
        erode_axis_kernel<<<nb, kBlock, 0, st>>>(mask, tmp, g, 1);
        SFC_TRY(launched("erode_axis_kernel"));
        erode_axis_kernel<<<nb, kBlock, 0, st>>>(tmp, valid, g, 0);
    } else {
        erode_axis_kernel<<<nb, kBlock, 0, st>>>(mask, valid, g, 2);
        SFC_TRY(launched("erode_axis_kernel"));
        erode_axis_kernel<<<nb, kBlock, 0, st>>>(valid, tmp, g, 1);
        SFC_TRY(launched("erode_axis_kernel"));
        erode_axis_kernel<<<nb, kBlock, 0, st>>>(tmp, valid, g, 0);
    }
    return launched("erode_axis_kernel");
}

sfc_status launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st) {
    if (n == 0) return SFC_OK;
    fill_u64_kernel<<<blocks_for(n), kBlock, 0, st>>>(p, n, v);
    return launched("fill_u64_kernel");
}

sfc_status launch_zero_f32(float* p, int64_t n, hipStream_t st) {
    if (n <= 0) return SFC_OK;
    zero_f32_kernel<<<blocks_for(n), kBlock, 0, st>>>(p, n);
    return launched("zero_f32_kernel");
}

sfc_status launch_pad_f32(const float* in, int64_t n, int64_t npad, float* out, hipStream_t st) {
    if (npad <= 0) return SFC_OK;
    pad_f32_kernel<<<blocks_for(npad), kBlock, 0, st>>>(in, n, npad, out);
    return launched("pad_f32_kernel");
}

sfc_status launch_u32_to_i64(const uint32_t* in, int64_t* out, int64_t n, hipStream_t st) {
    if (n == 0) return SFC_OK;
    u32_to_i64_kernel<<<blocks_for(n), kBlock, 0, st>>>(in, out, n);
    return launched("u32_to_i64_kernel");
}

}  // namespace sfc
