// Full scan of the dictionary in float32 (Section I: evaluate the masked L2
// cost of every fully known patch and keep the global minimum).
//
// Mapping on gfx950: candidates are walked along the fastest axis in "line
// tiles" of 64 * NX consecutive centres; each lane owns NX adjacent centres
// and reads their patch rows straight from memory (a row of NX candidates is
// K + NX - 1 voxels, shared through L1/L2). A block of QB queries is processed
// at a time: their targets and per-row known-masks are wave-uniform and come
// through scalar loads, so each known element costs one v_sub and one v_fma
// per lane per query per candidate. The per-candidate order (rows ascending,
// column ascending, channel ascending, fused multiply-add from +0) is exactly
// the definition's, so the cost bits are those of the definition. The
// (cost, id) minimum is kept per lane, reduced per wave, merged per query in
// LDS and then once per workgroup in global memory with a 64-bit atomic min
// on (cost bits << 32 | id), which is order independent.
//
// Two entry kernels share the body: one image, with an XCD-aware grid; and a
// batch of images of uneven size (each its own dictionary), a persistent grid
// walking (image, query block, tile chunk) work items.
#include <algorithm>

#include "batch.hpp"

namespace sfc {

namespace {

constexpr int kLanes = 256;
constexpr int kXcds = 8;
constexpr int kScanQB = 48;   // row-mask padding: a multiple of every variant's QB
// s_waitcnt with lgkmcnt(0) and the vector-memory and export counters at
// their maxima: waits for LDS, scalar-memory and message results only
constexpr int kWaitScalar = 0xC07F;
// vmcnt(0) with the export and LDS/scalar counters at their maxima
constexpr int kWaitVector = 0x0F70;

typedef const __attribute__((address_space(4))) float cfloat_as4;
typedef const __attribute__((address_space(4))) uint32_t cu32_as4;
// four floats at dword alignment
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

// Wave-uniform loads through the scalar cache.
__device__ inline float ldu(const float* p) { return *(cfloat_as4*)p; }
__device__ inline uint32_t ldu(const uint32_t* p) { return *(cu32_as4*)p; }


// Each lane owns NX adjacent candidates of a 64*NX-wide line tile; their
// patch rows are read straight from memory (L1/L2 resident), so waves run
// without barriers. The workgroup's four waves share the query batches and
// split its tiles; per batch, each wave keeps a per-lane running best
// (strict comparison in ascending id order keeps the lowest id), reduces it
// over the wave, and the workgroup merges the four results in LDS before one
// global atomic per query.
// Queries [q0, q1) against line tiles [tl0, tl1) of one image; the whole
// workgroup calls it (it synchronises). sred: LDS [4][QB].
// One known element's term: d*d fused into the sum (L2, Section II) or |d|
// added to it (L1, Section III.K), in the definition's order either way.
template <int NORM>
__device__ __forceinline__ float accum(float acc, float d) {
    if constexpr (NORM == 0) return __builtin_fmaf(d, d, acc);
    else return acc + __builtin_fabsf(d);
}

// Queries whose target rows are requested together: the largest power of
// two dividing QB whose rows (and masks) fit 16 scalar registers, so that
// short rows (one channel, small K) wait once per group instead of once per
// query.
constexpr int scan_group(int QB, int RW) {
    int g = 1;
    while (g * 2 <= QB && QB % (g * 2) == 0 && g * 2 * (RW + 1) <= 16) g *= 2;
    return g;
}

template <int ND, int K, int C, int QB, int NX, int NORM = 0>
__device__ __forceinline__ void scan_range(const ScanParams& p, int64_t q0, int64_t q1, int64_t tl0,
                                           int64_t tl1, uint64_t* sred) {
    constexpr int H = (K - 1) / 2;
    constexpr int ROWS = (ND == 2) ? K : K * K;
    constexpr int RW = K * C;
    constexpr int SEG = (K + NX - 1) * C;     // floats of one patch row for NX candidates
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    for (int64_t qb = q0; qb < q1; qb += QB) {
        uint32_t bcost[QB], bid[QB];
#pragma unroll
        for (int qi = 0; qi < QB; qi++) {
            bcost[qi] = 0xffffffffu;
            bid[qi] = 0xffffffffu;
        }
        for (int64_t tl = tl0 + wave; tl < tl1; tl += kLanes / 64) {
            int64_t line, x0;
            if (p.spans) {
                // 8 * NX spans per wave tile, NX adjacent candidates per lane
                static_assert(8 % NX == 0, "a lane's candidates lie in one span");
                const int64_t li = tl * (8 * NX) + (lane * NX) / 8;
                if (li < p.n_spans) {
                    const uint32_t sp = p.spans[li];
                    const uint32_t ln = sp / (uint32_t)p.spans_per_line;
                    line = ln;
                    x0 = (int64_t)(sp - ln * (uint32_t)p.spans_per_line) * 8 + (lane * NX) % 8;
                } else {
                    line = 0;            // past the list: no candidate
                    x0 = p.line_len;
                }
            } else {
                line = tl / p.tiles_per_line;
                x0 = (tl - line * p.tiles_per_line) * (64 * NX) + (int64_t)lane * NX;
            }
            int64_t base;
            if (ND == 2) {
                base = (line + H) * p.stride[0];
            } else {
                const uint32_t iy = (uint32_t)(p.shape[1] - 2 * H);
                const uint32_t z = (uint32_t)line / iy, y = (uint32_t)line - z * iy;
                base = ((int64_t)z + H) * p.stride[0] + ((int64_t)y + H) * p.stride[1];
            }
            const bool whole = x0 + NX <= p.line_len;   // all NX candidates inside the line
            float acc[QB][NX];
#pragma unroll
            for (int qi = 0; qi < QB; qi++)
#pragma unroll
                for (int j = 0; j < NX; j++) acc[qi][j] = 0.0f;
            for (int r = 0; r < ROWS; r++) {
                const uint32_t* mrb = p.rowmask + (int64_t)r * p.qpad + qb;
                int64_t roff;
                if (ND == 2) roff = (int64_t)(r - H) * p.stride[0];
                else roff = (int64_t)(r / K - H) * p.stride[0] + (int64_t)(r % K - H) * p.stride[1];
                const float* vp = p.vol + (base + roff + x0) * C;
                float v[SEG];
                if (whole) {
                    // 16-byte loads at 4-byte alignment (global loads of
                    // this width need only dword alignment)
                    const f4u* vp4 = reinterpret_cast<const f4u*>(vp);
#pragma unroll
                    for (int i = 0; i < SEG / 4; i++) {
                        const f4u x = vp4[i];
                        v[4 * i] = x.x;
                        v[4 * i + 1] = x.y;
                        v[4 * i + 2] = x.z;
                        v[4 * i + 3] = x.w;
                    }
#pragma unroll
                    for (int i = (SEG / 4) * 4; i < SEG; i++) v[i] = vp[i];
                } else {
#pragma unroll
                    for (int i = 0; i < SEG; i++)
                        v[i] = (x0 + i / C < p.shape[ND - 1]) ? vp[i] : 0.0f;
                }
                // the row's loads are complete before any query's pixels,
                // so the conditional pixel blocks carry no waits of their own
                __builtin_amdgcn_s_waitcnt(kWaitVector);
                const float* tb = p.t + (qb * ROWS + r) * RW;
                // The query rows come through scalar loads, which return out
                // of order, so a wait covers every one in flight. Queries go
                // in groups of G (G > 1 for short rows): the next group's
                // rows are requested only after the current group's have
                // arrived, and are consumed while that request is in flight.
                // (Targets are padded to the query block: all in bounds.)
                constexpr int G = scan_group(QB, RW);
                float tc[G][RW];
                uint32_t mc[G];
#pragma unroll
                for (int k = 0; k < G; k++) {
#pragma unroll
                    for (int i = 0; i < RW; i++) tc[k][i] = ldu(tb + k * ROWS * RW + i);
                    mc[k] = ldu(mrb + k);
                }
#pragma unroll
                for (int q0g = 0; q0g < QB; q0g += G) {
                    __builtin_amdgcn_s_waitcnt(kWaitScalar);
                    float tn[G][RW];
                    uint32_t mn[G];
                    if (q0g + G < QB) {
#pragma unroll
                        for (int k = 0; k < G; k++) {
#pragma unroll
                            for (int i = 0; i < RW; i++)
                                tn[k][i] = ldu(tb + (q0g + G + k) * ROWS * RW + i);
                            mn[k] = ldu(mrb + q0g + G + k);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < G; k++) {
                        const int qi = q0g + k;
                        const uint32_t mr = mc[k];
                        // known pixels of the row only, each updating the NX
                        // accumulators in place (a full row takes every branch)
                        if (mr != 0) {
#pragma unroll
                            for (int dx = 0; dx < K; dx++) {
                                if (mr & (1u << dx)) {
#pragma unroll
                                    for (int j = 0; j < NX; j++)
#pragma unroll
                                        for (int ch = 0; ch < C; ch++) {
                                            const float d = tc[k][dx * C + ch] - v[(j + dx) * C + ch];
                                            acc[qi][j] = accum<NORM>(acc[qi][j], d);
                                        }
                                }
                            }
                        }
                    }
                    if (q0g + G < QB) {
#pragma unroll
                        for (int k = 0; k < G; k++) {
#pragma unroll
                            for (int i = 0; i < RW; i++) tc[k][i] = tn[k][i];
                            mc[k] = mn[k];
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NX; j++) {
                const int64_t xi = x0 + j;
                const uint32_t cid = (uint32_t)(base + xi + H);
                if (xi < p.line_len && p.valid[cid]) {
#pragma unroll
                    for (int qi = 0; qi < QB; qi++) {
                        const uint32_t cb = __float_as_uint(acc[qi][j]);
                        if (cb < bcost[qi]) {
                            bcost[qi] = cb;
                            bid[qi] = cid;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int qi = 0; qi < QB; qi++) {
            uint64_t pk = ((uint64_t)bcost[qi] << 32) | bid[qi];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const uint64_t o = (uint64_t)__shfl_xor((long long)pk, off, 64);
                pk = o < pk ? o : pk;
            }
            if (lane == 0) sred[wave * QB + qi] = pk;
        }
        __syncthreads();
        if (tid < QB && qb + tid < q1) {
            uint64_t best = sred[tid];
#pragma unroll
            for (int w = 1; w < kLanes / 64; w++)
                best = sred[w * QB + tid] < best ? sred[w * QB + tid] : best;
            if ((best >> 32) != 0xffffffffull)
                atomicMin((unsigned long long*)&p.best[qb + tid], (unsigned long long)best);
        }
        __syncthreads();
    }
}

template <int ND, int K, int C, int QB, int NX, int NORM>
__global__ __launch_bounds__(kLanes) void scan_fp32_kernel(ScanParams p) {
    __shared__ uint64_t sred[(kLanes / 64) * QB];
    // XCD-aware mapping: workgroups are dispatched to the 8 XCDs round-robin,
    // so block b runs on XCD b % 8. Each XCD gets a contiguous band of tile
    // chunks. Its slots walk groups of q_group query splits (targets of a
    // group fit the XCD's L2 next to a chunk's patch rows); within a group
    // every chunk of the band in turn, and within a chunk the group's splits
    // fastest. So the workgroups resident on an XCD at one time walk the same
    // chunk's tiles (each with its own queries): a patch row comes from HBM
    // about once per group and XCD, a target once per XCD.
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % kXcds, slot = b / kXcds;
    const int64_t per_group = p.chunks_per_xcd * p.q_group;
    const int64_t qg = slot / per_group, rem = slot - qg * per_group;
    const int64_t chunk = xcd * p.chunks_per_xcd + rem / p.q_group;
    const int64_t qs = qg * p.q_group + rem % p.q_group;
    if (qs >= p.q_splits || chunk >= p.n_chunks) return;
    const int64_t q0 = qs * p.q_per_wg;
    const int64_t q1 = min(p.Q, q0 + p.q_per_wg);
    if (q0 >= q1) return;
    const int64_t tl0 = chunk * p.tiles_per_wg;
    const int64_t tl1 = min(p.n_tiles, tl0 + p.tiles_per_wg);
    scan_range<ND, K, C, QB, NX, NORM>(p, q0, q1, tl0, tl1, sred);
}

// ---- batches of 2D images
// (QB, NX) of a batch shape set for a channel count
constexpr int batch_qb(int shape, int C) { return shape == 1 ? 8 : 16; }
constexpr int batch_nx(int shape, int C) {
    return shape == 2 ? (C == 1 ? 4 : 2) : (C == 1 ? 8 : 4);
}

template <int K, int SHAPE>
__global__ __launch_bounds__(kLanes) void scan_batch_kernel(const ScanParams* __restrict__ imgs,
                                                            const int32_t* __restrict__ img_c,
                                                            const BatchItem* __restrict__ items,
                                                            int64_t n_items) {
    __shared__ uint64_t sred[(kLanes / 64) * 16];
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const BatchItem w = items[it];
        const ScanParams p = imgs[w.image];
        const int C = img_c[w.image];
        if (C == 1)
            scan_range<2, K, 1, batch_qb(SHAPE, 1), batch_nx(SHAPE, 1)>(p, w.q0, w.q1, w.tl0,
                                                                         w.tl1, sred);
        else if (C == 2)
            scan_range<2, K, 2, batch_qb(SHAPE, 2), batch_nx(SHAPE, 2)>(p, w.q0, w.q1, w.tl0,
                                                                         w.tl1, sred);
        else
            scan_range<2, K, 3, batch_qb(SHAPE, 3), batch_nx(SHAPE, 3)>(p, w.q0, w.q1, w.tl0,
                                                                         w.tl1, sred);
    }
}

// Padded targets, row masks and cleared results of every image of a batch:
// one thread per (padded query, patch row). Padded query g belongs to the
// image i with pad_start[i] <= g < pad_start[i + 1].
__global__ void batch_prep_kernel(const float* __restrict__ targets, const uint8_t* __restrict__ masks,
                                  const BatchMeta* __restrict__ meta, const int64_t* __restrict__ pad_start,
                                  int n_images, int K, int64_t total_pad, float* __restrict__ tpad,
                                  uint32_t* __restrict__ rowmask, uint64_t* __restrict__ best) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total_pad * K) return;
    const int64_t g = e / K;
    const int r = (int)(e - g * K);
    int lo = 0, hi = n_images - 1;
    while (lo < hi) {   // last image whose padded range starts at or before g
        const int mid = (lo + hi + 1) >> 1;
        if (pad_start[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const BatchMeta m = meta[lo];
    const int64_t ql = g - pad_start[lo];
    const int C = m.C, RW = K * C;
    float* dst = tpad + m.tpad_off + (ql * K + r) * RW;
    uint32_t bits = 0;
    if (ql < m.Q) {
        const int64_t q = m.q_off + ql;
        const float* src = targets + m.t_off + (ql * K + r) * RW;
        for (int i = 0; i < RW; i++) dst[i] = src[i];
        const uint8_t* mk = masks + (q * K + r) * K;
        for (int dx = 0; dx < K; dx++)
            if (mk[dx]) bits |= 1u << dx;
        if (r == 0) best[q] = ~0ull;
    } else {
        for (int i = 0; i < RW; i++) dst[i] = 0.0f;
    }
    rowmask[m.rm_off + (int64_t)r * m.qpad + ql] = bits;
}

// rowmask[r][q] bit dx = target_masks[q][r*K + dx]; queries Q..qpad-1 get 0.
__global__ void pack_rowmask_kernel(const uint8_t* __restrict__ m, int64_t Q, int64_t qpad,
                                    int rows, int K, uint32_t* __restrict__ rowmask) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= qpad * rows) return;
    const int64_t r = i / qpad, q = i - r * qpad;
    uint32_t bits = 0;
    if (q < Q) {
        const uint8_t* src = m + (q * rows + r) * K;
        for (int dx = 0; dx < K; dx++)
            if (src[dx]) bits |= 1u << dx;
    }
    rowmask[i] = bits;
}

__global__ void unpack_best_kernel(const uint64_t* __restrict__ best, int64_t Q,
                                   int64_t* __restrict__ id, float* __restrict__ cost) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const uint64_t b = best[q];
    if (b == ~0ull) {
        id[q] = -1;
        cost[q] = __builtin_inff();
    } else {
        id[q] = (int64_t)(b & 0xffffffffull);
        cost[q] = __uint_as_float((uint32_t)(b >> 32));
    }
}

// flags[s] = 1 when span s (positions 8 (s % spl) .. + 7 of interior line
// s / spl) holds a dictionary centre
__global__ void span_flags_kernel(const uint8_t* __restrict__ valid, int nd, int64_t st0,
                                  int64_t st1, int64_t iy, int H, int64_t line_len, int64_t spl,
                                  int64_t slots, uint8_t* __restrict__ flags) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= slots) return;
    const int64_t line = s / spl, x8 = s - line * spl;
    int64_t base;
    if (nd == 2) {
        base = (line + H) * st0;
    } else {
        const int64_t z = line / iy, y = line - z * iy;
        base = (z + H) * st0 + (y + H) * st1;
    }
    uint8_t any = 0;
    const int64_t x1 = min(x8 * 8 + 8, line_len);
    for (int64_t x = x8 * 8; x < x1; x++) any |= valid[base + x + H];
    flags[s] = any ? 1 : 0;
}

using ScanFn = void (*)(ScanParams);

struct ScanEntry {
    int nd, K, C;
    int qb, nx;
    ScanFn fn;
    ScanFn fn_l1;   // the L1 cost with this shape (default shapes only)
};

// (QB queries per pass, NX candidates per lane) shapes per (ndim, K, C); the
// first entry of a shape is its default, the others are candidates for the
// autotuner.
#define SFC_SCAN(ND, K, C, QB, NX) {ND, K, C, QB, NX, scan_fp32_kernel<ND, K, C, QB, NX, 0>, nullptr}
// a default shape: also instantiated for the L1 cost
#define SFC_SCAN1(ND, K, C, QB, NX)                                                           \
    {ND, K, C, QB, NX, scan_fp32_kernel<ND, K, C, QB, NX, 0>, scan_fp32_kernel<ND, K, C, QB, NX, 1>}
const ScanEntry kScanTable[] = {
    SFC_SCAN1(2, 3, 1, 16, 8), SFC_SCAN1(2, 3, 2, 16, 8), SFC_SCAN1(2, 3, 3, 16, 8),
    SFC_SCAN1(2, 5, 1, 16, 8), SFC_SCAN1(2, 5, 2, 16, 4), SFC_SCAN1(2, 5, 3, 16, 4),
    SFC_SCAN1(2, 7, 1, 16, 8), SFC_SCAN1(2, 7, 2, 16, 4), SFC_SCAN1(2, 7, 3, 16, 4),
    SFC_SCAN1(2, 9, 1, 16, 8), SFC_SCAN(2, 9, 1, 16, 4), SFC_SCAN(2, 9, 1, 8, 8),
    SFC_SCAN1(2, 9, 2, 16, 4),
    SFC_SCAN1(2, 9, 3, 8, 4), SFC_SCAN(2, 9, 3, 8, 8), SFC_SCAN(2, 9, 3, 16, 4),
    SFC_SCAN(2, 9, 3, 16, 2), SFC_SCAN(2, 9, 3, 12, 4),
    SFC_SCAN1(2, 11, 1, 16, 4), SFC_SCAN1(2, 11, 3, 16, 2),
    SFC_SCAN1(2, 13, 1, 16, 4), SFC_SCAN1(2, 13, 3, 8, 2),
    SFC_SCAN1(3, 3, 1, 16, 8), SFC_SCAN1(3, 3, 2, 16, 8),
    SFC_SCAN1(3, 5, 1, 8, 8), SFC_SCAN(3, 5, 1, 16, 8), SFC_SCAN(3, 5, 1, 16, 4),
    SFC_SCAN1(3, 5, 2, 16, 4),
    SFC_SCAN1(3, 7, 1, 8, 8), SFC_SCAN(3, 7, 1, 16, 4), SFC_SCAN(3, 7, 1, 16, 8),
};

// One shape per (ndim, K, C) for one or two queries (the fill loop asks for
// a single target): QB = 2, so a lone query costs two query slots of work
// instead of a whole query block. Not offered to the autotuner.
const ScanEntry kScanSmall[] = {
    SFC_SCAN(2, 3, 1, 2, 8), SFC_SCAN(2, 3, 2, 2, 8), SFC_SCAN(2, 3, 3, 2, 8),
    SFC_SCAN(2, 5, 1, 2, 8), SFC_SCAN(2, 5, 2, 2, 8), SFC_SCAN(2, 5, 3, 2, 8),
    SFC_SCAN(2, 7, 1, 2, 8), SFC_SCAN(2, 7, 2, 2, 8), SFC_SCAN(2, 7, 3, 2, 8),
    SFC_SCAN(2, 9, 1, 2, 8), SFC_SCAN(2, 9, 2, 2, 8), SFC_SCAN(2, 9, 3, 2, 8),
    SFC_SCAN(2, 11, 1, 2, 8), SFC_SCAN(2, 11, 3, 2, 4),
    SFC_SCAN(2, 13, 1, 2, 8), SFC_SCAN(2, 13, 3, 2, 4),
    SFC_SCAN(3, 3, 1, 2, 8), SFC_SCAN(3, 3, 2, 2, 8),
    SFC_SCAN(3, 5, 1, 2, 8), SFC_SCAN(3, 5, 2, 2, 8),
    SFC_SCAN(3, 7, 1, 2, 8),
};

const ScanEntry* scan_entry_small(int nd, int K, int C) {
    for (const auto& e : kScanSmall)
        if (e.nd == nd && e.K == K && e.C == C) return &e;
    return nullptr;
}

// variant v (0 = default) of a shape, or null
const ScanEntry* scan_entry(int nd, int K, int C, int v) {
    int k = 0;
    for (const auto& e : kScanTable)
        if (e.nd == nd && e.K == K && e.C == C) {
            if (k == v) return &e;
            k++;
        }
    return nullptr;
}

// the shape of (nd, K, C) that has an L1 kernel, or null
const ScanEntry* scan_entry_l1(int nd, int K, int C) {
    for (const auto& e : kScanTable)
        if (e.nd == nd && e.K == K && e.C == C && e.fn_l1) return &e;
    return nullptr;
}

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Workgroups of a table entry resident on the whole device at once (its
// occupancy per CU from its register use, times the CUs), cached per entry.
int64_t resident_slots(const ScanEntry* e) {
    constexpr int kMain = sizeof(kScanTable) / sizeof(kScanTable[0]);
    constexpr int kEntries = kMain + sizeof(kScanSmall) / sizeof(kScanSmall[0]);
    static int64_t slots[kEntries] = {0};
    const bool small = e >= kScanSmall && e < kScanSmall + (kEntries - kMain);
    const int idx = small ? kMain + (int)(e - kScanSmall) : (int)(e - kScanTable);
    if (slots[idx] == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(e->fn),
                                                         kLanes, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        slots[idx] = (int64_t)per_cu * cus;
    }
    return slots[idx];
}

}  // namespace

bool scan_supported(int nd, int K, int C) { return scan_entry(nd, K, C, 0) != nullptr; }

int scan_variants(int nd, int K, int C) {
    int k = 0;
    while (scan_entry(nd, K, C, k)) k++;
    return k;
}

int64_t scan_qpad(int64_t Q) { return ((Q + kScanQB - 1) / kScanQB) * kScanQB; }  // multiple of every QB

namespace {
void scan_lines(const Grid& g, int64_t* n_lines, int64_t* line_len) {
    int64_t nl = 1;
    for (int i = 0; i < g.nd - 1; i++) nl *= (g.shape[i] - 2 * g.h);
    *n_lines = nl;
    *line_len = g.shape[g.nd - 1] - 2 * g.h;
}
}  // namespace

int64_t scan_span_slots(const Grid& g) {
    int64_t nl, len;
    scan_lines(g, &nl, &len);
    if (nl <= 0 || len <= 0) return 0;
    return nl * ((len + 7) / 8);
}

sfc_status launch_span_flags(const Grid& g, const uint8_t* valid, uint8_t* flags, hipStream_t st) {
    int64_t nl, len;
    scan_lines(g, &nl, &len);
    const int64_t slots = scan_span_slots(g);
    if (slots == 0) return SFC_OK;
    span_flags_kernel<<<blocks_for(slots), 256, 0, st>>>(
        valid, g.nd, g.stride[0], g.nd == 3 ? g.stride[1] : 0,
        g.nd == 3 ? g.shape[1] - 2 * g.h : 1, g.h, len, (len + 7) / 8, slots, flags);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "span_flags_kernel");
}

sfc_status launch_pack_rowmask(const uint8_t* m, const Grid& g, int64_t Q, uint32_t* rowmask,
                               hipStream_t st) {
    if (Q == 0) return SFC_OK;
    const int64_t qpad = scan_qpad(Q);
    pack_rowmask_kernel<<<blocks_for(qpad * g.rows), 256, 0, st>>>(m, Q, qpad, g.rows, g.K,
                                                                   rowmask);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "pack_rowmask_kernel");
}

sfc_status launch_unpack_best(const uint64_t* best, int64_t Q, int64_t* id, float* cost,
                              hipStream_t st) {
    if (Q == 0) return SFC_OK;
    unpack_best_kernel<<<blocks_for(Q), 256, 0, st>>>(best, Q, id, cost);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "unpack_best_kernel");
}

sfc_status launch_scan_fp32(const Grid& g, const ScanArgs& a, hipStream_t st) {
    if (a.Q == 0) return SFC_OK;
    const ScanEntry* ent;
    if (a.norm == 1) {
        ent = scan_entry_l1(g.nd, g.K, g.C);
    } else {
        ent = a.Q <= 2 ? scan_entry_small(g.nd, g.K, g.C) : nullptr;
        if (!ent) ent = scan_entry(g.nd, g.K, g.C, a.variant);
        if (!ent) ent = scan_entry(g.nd, g.K, g.C, 0);
    }
    if (!ent)
        return fail(SFC_EUNSUPPORTED, "float32 scan: no kernel for this (ndim, K, channels)");
    const ScanFn fn = a.norm == 1 ? ent->fn_l1 : ent->fn;
    ScanParams p{};
    p.vol = a.vol;
    p.valid = a.valid;
    p.t = a.t;
    p.rowmask = a.rowmask;
    p.best = a.best;
    p.Q = a.Q;
    for (int i = 0; i < g.nd; i++) {
        p.shape[i] = g.shape[i];
        p.stride[i] = g.stride[i];
    }
    int64_t n_lines = 1;
    for (int i = 0; i < g.nd - 1; i++) n_lines *= (g.shape[i] - 2 * g.h);
    p.line_len = g.shape[g.nd - 1] - 2 * g.h;
    if (n_lines <= 0 || p.line_len <= 0) return SFC_OK;
    const int64_t tw = 64 * ent->nx;   // candidates per wave tile
    p.tiles_per_line = (p.line_len + tw - 1) / tw;
    p.n_tiles = n_lines * p.tiles_per_line;
    if (a.spans && a.n_spans > 0) {
        // the tiles walk the spans that hold a centre (8 * NX per tile)
        p.spans = a.spans;
        p.n_spans = a.n_spans;
        p.spans_per_line = (p.line_len + 7) / 8;
        p.n_tiles = (a.n_spans + 8 * ent->nx - 1) / (8 * ent->nx);
    }
    // queries per workgroup (one block of QB unless the caller asks for
    // more), then tiles per workgroup so that the grid holds about 16 rounds
    // of the workgroups resident at once (with equal workgroups the last,
    // partly filled round costs a few percent instead of up to a third of
    // the launch), in a multiple of 8 chunks so the XCDs' bands are equal
    int64_t qpw = a.query_block > 0 ? a.query_block : ent->qb;
    qpw = ((qpw + ent->qb - 1) / ent->qb) * ent->qb;
    if (qpw > a.Q) qpw = ((a.Q + ent->qb - 1) / ent->qb) * ent->qb;
    p.q_per_wg = qpw;
    p.qpad = scan_qpad(a.Q);
    const int64_t qsplit = (a.Q + qpw - 1) / qpw;
    const int64_t target = 16 * resident_slots(ent);
    int64_t want = (target + qsplit - 1) / qsplit;              // chunks
    want = ((want + kXcds - 1) / kXcds) * kXcds;
    int64_t tpw = (p.n_tiles + want - 1) / want;
    tpw = ((tpw + 3) / 4) * 4;
    if (tpw < 4) tpw = 4;
    p.tiles_per_wg = tpw;
    const int64_t chunks = (p.n_tiles + tpw - 1) / tpw;
    p.n_chunks = chunks;
    p.chunks_per_xcd = (chunks + kXcds - 1) / kXcds;
    p.q_splits = qsplit;
    // query splits per group: their targets and row masks within 2 MiB,
    // the groups as equal as the split count allows
    const int64_t split_bytes = qpw * ((int64_t)g.Kd * g.C + g.rows) * 4;
    const int64_t most = std::max<int64_t>(1, std::min<int64_t>(qsplit, (int64_t(2) << 20) / split_bytes));
    const int64_t groups = (qsplit + most - 1) / most;
    p.q_group = (qsplit + groups - 1) / groups;
    const int64_t nblocks = kXcds * p.chunks_per_xcd * p.q_group * groups;
    if (nblocks > 0x7fffffffLL) return fail(SFC_EUNSUPPORTED, "float32 scan: grid too large");
    hipLaunchKernelGGL(fn, dim3((unsigned)nblocks), dim3(kLanes), 0, st, p);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "scan_fp32_kernel");
}

sfc_status launch_batch_prep(const float* targets, const uint8_t* masks, const BatchMeta* meta,
                             const int64_t* pad_start, int n_images, int K, int64_t total_pad,
                             float* tpad, uint32_t* rowmask, uint64_t* best, hipStream_t st) {
    if (total_pad == 0) return SFC_OK;
    batch_prep_kernel<<<blocks_for(total_pad * K), 256, 0, st>>>(targets, masks, meta, pad_start,
                                                                n_images, K, total_pad, tpad,
                                                                rowmask, best);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "batch_prep_kernel");
}

bool batch_scan_supported(int K) { return K == 5 || K == 7 || K == 9 || K == 11; }

sfc_status launch_batch_scan(int K, int shape, const ScanParams* imgs, const int32_t* img_c,
                             const BatchItem* items, int64_t n_items, unsigned grid,
                             hipStream_t st) {
    if (n_items == 0) return SFC_OK;
    using Fn = void (*)(const ScanParams*, const int32_t*, const BatchItem*, int64_t);
    Fn fn = nullptr;
#define SFC_BATCH_K(KK)                                                  \
    if (K == KK) {                                                       \
        fn = shape == 1   ? scan_batch_kernel<KK, 1>                      \
             : shape == 2 ? scan_batch_kernel<KK, 2>                      \
                          : scan_batch_kernel<KK, 0>;                     \
    }
    SFC_BATCH_K(5)
    SFC_BATCH_K(7)
    SFC_BATCH_K(9)
    SFC_BATCH_K(11)
#undef SFC_BATCH_K
    if (!fn) return fail(SFC_EUNSUPPORTED, "batched scan: K must be 5, 7, 9 or 11");
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kLanes), 0, st, imgs, img_c, items, n_items);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "scan_batch_kernel");
}

ScanParams batch_image_params(const Grid& g, const float* vol, const uint8_t* valid,
                              const uint32_t* spans, int64_t n_spans, const float* t,
                              const uint32_t* rowmask, uint64_t* best, int64_t Q, int64_t qpad,
                              int shape, int64_t* n_tiles) {
    ScanParams p{};
    p.vol = vol;
    p.valid = valid;
    p.t = t;
    p.rowmask = rowmask;
    p.best = best;
    p.Q = Q;
    for (int i = 0; i < g.nd; i++) {
        p.shape[i] = g.shape[i];
        p.stride[i] = g.stride[i];
    }
    const int nx = shape == 2 ? (g.C == 1 ? 4 : 2) : (g.C == 1 ? 8 : 4);
    p.line_len = g.shape[g.nd - 1] - 2 * g.h;
    const int64_t lines = g.shape[0] - 2 * g.h;
    p.tiles_per_line = p.line_len > 0 ? (p.line_len + 64 * nx - 1) / (64 * nx) : 0;
    p.n_tiles = lines > 0 ? lines * p.tiles_per_line : 0;
    if (spans && n_spans > 0 && p.n_tiles > 0) {
        p.spans = spans;
        p.n_spans = n_spans;
        p.spans_per_line = (p.line_len + 7) / 8;
        p.n_tiles = (n_spans + 8 * nx - 1) / (8 * nx);
    }
    p.qpad = qpad;
    *n_tiles = p.n_tiles;
    return p;
}

int batch_query_block(int shape) { return shape == 1 ? 8 : 16; }

}  // namespace sfc
