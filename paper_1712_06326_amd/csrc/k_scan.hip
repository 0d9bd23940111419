// Full scan of the dictionary in float32 (Section I: evaluate the masked L2
// cost of every fully known patch and keep the global minimum).
//
// Mapping on gfx950: one workgroup of 256 lanes owns a "line tile" of 256
// consecutive candidate centres along the fastest axis and stages the K^(nd-1)
// volume rows those patches touch in LDS. Each lane is one candidate. A block
// of QB queries is processed at a time: their targets and per-row known-masks
// are wave-uniform and come through scalar loads, so each known element costs
// one v_sub and one v_fma per lane per query, with the LDS row values reused
// across the QB accumulators. The per-candidate order (rows ascending, column
// ascending, channel ascending, fused multiply-add from +0) is exactly the
// reference cost order, so the cost bits are those of the definition. The
// (cost, id) minimum is reduced per wave, merged per query in LDS and then
// once per workgroup in global memory with a 64-bit atomic min on
// (cost bits << 32 | id), which is order independent.
#include "common.hpp"

namespace sfc {

namespace {

constexpr int kLanes = 256;
constexpr int kXcds = 8;
constexpr int kScanQB = 48;   // row-mask padding: a multiple of every variant's QB

typedef const __attribute__((address_space(4))) float cfloat_as4;
typedef const __attribute__((address_space(4))) uint32_t cu32_as4;

// Wave-uniform loads through the scalar cache.
__device__ inline float ldu(const float* p) { return *(cfloat_as4*)p; }
__device__ inline uint32_t ldu(const uint32_t* p) { return *(cu32_as4*)p; }

struct ScanParams {
    const float* vol;
    const uint8_t* valid;
    const float* t;
    const uint32_t* rowmask;
    uint64_t* best;
    int64_t Q;
    int64_t shape[kMaxDims];
    int64_t stride[kMaxDims];
    int64_t line_len;        // interior extent along the fastest axis
    int64_t tiles_per_line;
    int64_t n_tiles;
    int64_t tiles_per_wg;
    int64_t q_per_wg;
    int64_t qpad;            // row-mask stride (queries padded to the block size)
    int64_t n_chunks, chunks_per_xcd, q_splits;
};

// Each lane owns NX adjacent candidates of a 64*NX-wide line tile; their
// patch rows are read straight from memory (L1/L2 resident), so waves run
// without barriers. The workgroup's four waves share the query batches and
// split its tiles; per batch, each wave keeps a per-lane running best
// (strict comparison in ascending id order keeps the lowest id), reduces it
// over the wave, and the workgroup merges the four results in LDS before one
// global atomic per query.
template <int ND, int K, int C, int QB, int NX>
__global__ __launch_bounds__(kLanes) void scan_fp32_kernel(ScanParams p) {
    constexpr int H = (K - 1) / 2;
    constexpr int ROWS = (ND == 2) ? K : K * K;
    constexpr int RW = K * C;
    constexpr int SEG = (K + NX - 1) * C;     // floats of one patch row for NX candidates
    __shared__ uint64_t sred[kLanes / 64][QB];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    // XCD-aware mapping: workgroups are dispatched to the 8 XCDs round-robin,
    // so block b runs on XCD b % 8. Each XCD gets a contiguous band of tile
    // chunks (all query splits of it), keeping its band of the volume in
    // that XCD's L2.
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % kXcds, slot = b / kXcds;
    const int64_t chunk = xcd * p.chunks_per_xcd + slot % p.chunks_per_xcd;
    const int64_t qs = slot / p.chunks_per_xcd;
    if (chunk >= p.n_chunks || qs >= p.q_splits) return;
    const int64_t q0 = qs * p.q_per_wg;
    const int64_t q1 = min(p.Q, q0 + p.q_per_wg);
    if (q0 >= q1) return;
    const int64_t tl0 = chunk * p.tiles_per_wg;
    const int64_t tl1 = min(p.n_tiles, tl0 + p.tiles_per_wg);

    for (int64_t qb = q0; qb < q1; qb += QB) {
        uint32_t bcost[QB], bid[QB];
#pragma unroll
        for (int qi = 0; qi < QB; qi++) {
            bcost[qi] = 0xffffffffu;
            bid[qi] = 0xffffffffu;
        }
        for (int64_t tl = tl0 + wave; tl < tl1; tl += kLanes / 64) {
            const int64_t line = tl / p.tiles_per_line;
            const int64_t x0 = (tl - line * p.tiles_per_line) * (64 * NX) + (int64_t)lane * NX;
            int64_t base;
            if (ND == 2) {
                base = (line + H) * p.stride[0];
            } else {
                const int64_t iy = p.shape[1] - 2 * H;
                const int64_t z = line / iy, y = line - z * iy;
                base = (z + H) * p.stride[0] + (y + H) * p.stride[1];
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
#pragma unroll
                    for (int i = 0; i < SEG; i++) v[i] = vp[i];
                } else {
#pragma unroll
                    for (int i = 0; i < SEG; i++)
                        v[i] = (x0 + i / C < p.shape[ND - 1]) ? vp[i] : 0.0f;
                }
                const float* tb = p.t + (qb * ROWS + r) * RW;
#pragma unroll
                for (int qi = 0; qi < QB; qi++) {
                    // targets are padded to the query block: both loads are in
                    // bounds and issue together before one wait
                    float tr[RW];
#pragma unroll
                    for (int i = 0; i < RW; i++) tr[i] = ldu(tb + qi * ROWS * RW + i);
                    const uint32_t mr = ldu(mrb + qi);
                    if (mr == 0) continue;
                    if (mr == (1u << K) - 1u) {
#pragma unroll
                        for (int j = 0; j < NX; j++)
#pragma unroll
                            for (int i = 0; i < RW; i++) {
                                const float d = tr[i] - v[j * C + i];
                                acc[qi][j] = __builtin_fmaf(d, d, acc[qi][j]);
                            }
                    } else {
#pragma unroll
                        for (int dx = 0; dx < K; dx++) {
                            if (mr & (1u << dx)) {
#pragma unroll
                                for (int j = 0; j < NX; j++)
#pragma unroll
                                    for (int ch = 0; ch < C; ch++) {
                                        const float d = tr[dx * C + ch] - v[(j + dx) * C + ch];
                                        acc[qi][j] = __builtin_fmaf(d, d, acc[qi][j]);
                                    }
                            }
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
            if (lane == 0) sred[wave][qi] = pk;
        }
        __syncthreads();
        if (tid < QB && qb + tid < q1) {
            uint64_t best = sred[0][tid];
#pragma unroll
            for (int w = 1; w < kLanes / 64; w++) best = sred[w][tid] < best ? sred[w][tid] : best;
            if ((best >> 32) != 0xffffffffull)
                atomicMin((unsigned long long*)&p.best[qb + tid], (unsigned long long)best);
        }
        __syncthreads();
    }
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

using ScanFn = void (*)(ScanParams);

struct ScanEntry {
    int nd, K, C;
    int qb, nx;
    ScanFn fn;
};

// (QB queries per pass, NX candidates per lane) shapes per (ndim, K, C); the
// first entry of a shape is its default, the others are candidates for the
// autotuner.
#define SFC_SCAN(ND, K, C, QB, NX) {ND, K, C, QB, NX, scan_fp32_kernel<ND, K, C, QB, NX>}
const ScanEntry kScanTable[] = {
    SFC_SCAN(2, 3, 1, 16, 8), SFC_SCAN(2, 3, 2, 16, 8), SFC_SCAN(2, 3, 3, 16, 8),
    SFC_SCAN(2, 5, 1, 16, 8), SFC_SCAN(2, 5, 2, 16, 4), SFC_SCAN(2, 5, 3, 16, 4),
    SFC_SCAN(2, 7, 1, 16, 8), SFC_SCAN(2, 7, 2, 16, 4), SFC_SCAN(2, 7, 3, 16, 4),
    SFC_SCAN(2, 9, 1, 16, 8), SFC_SCAN(2, 9, 1, 16, 4), SFC_SCAN(2, 9, 1, 8, 8),
    SFC_SCAN(2, 9, 2, 16, 4),
    SFC_SCAN(2, 9, 3, 16, 4), SFC_SCAN(2, 9, 3, 8, 4), SFC_SCAN(2, 9, 3, 16, 2),
    SFC_SCAN(2, 9, 3, 8, 8), SFC_SCAN(2, 9, 3, 12, 4),
    SFC_SCAN(2, 11, 1, 16, 4), SFC_SCAN(2, 11, 3, 16, 2),
    SFC_SCAN(2, 13, 1, 16, 4), SFC_SCAN(2, 13, 3, 8, 2),
    SFC_SCAN(3, 3, 1, 16, 8), SFC_SCAN(3, 3, 2, 16, 8),
    SFC_SCAN(3, 5, 1, 16, 8), SFC_SCAN(3, 5, 1, 16, 4), SFC_SCAN(3, 5, 1, 8, 8),
    SFC_SCAN(3, 5, 2, 16, 4),
    SFC_SCAN(3, 7, 1, 16, 4), SFC_SCAN(3, 7, 1, 16, 8), SFC_SCAN(3, 7, 1, 8, 8),
};

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

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

bool scan_supported(int nd, int K, int C) { return scan_entry(nd, K, C, 0) != nullptr; }

int scan_variants(int nd, int K, int C) {
    int k = 0;
    while (scan_entry(nd, K, C, k)) k++;
    return k;
}

int64_t scan_qpad(int64_t Q) { return ((Q + kScanQB - 1) / kScanQB) * kScanQB; }  // multiple of every QB

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
    const ScanEntry* ent = scan_entry(g.nd, g.K, g.C, a.variant);
    if (!ent) ent = scan_entry(g.nd, g.K, g.C, 0);
    if (!ent)
        return fail(SFC_EUNSUPPORTED, "float32 scan: no kernel for this (ndim, K, channels)");
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
    // queries per workgroup, then tiles per workgroup so that the grid holds
    // about 4096 workgroups (16 per CU)
    int64_t qpw = a.query_block > 0 ? a.query_block : 512;
    qpw = ((qpw + ent->qb - 1) / ent->qb) * ent->qb;
    if (qpw > a.Q) qpw = ((a.Q + ent->qb - 1) / ent->qb) * ent->qb;
    p.q_per_wg = qpw;
    p.qpad = scan_qpad(a.Q);
    const int64_t qsplit = (a.Q + qpw - 1) / qpw;
    int64_t tpw = (p.n_tiles * qsplit + 4095) / 4096;
    tpw = ((tpw + 3) / 4) * 4;
    if (tpw < 4) tpw = 4;
    p.tiles_per_wg = tpw;
    const int64_t chunks = (p.n_tiles + tpw - 1) / tpw;
    p.n_chunks = chunks;
    p.chunks_per_xcd = (chunks + kXcds - 1) / kXcds;
    p.q_splits = qsplit;
    const int64_t nblocks = kXcds * p.chunks_per_xcd * qsplit;
    if (nblocks > 0x7fffffffLL) return fail(SFC_EUNSUPPORTED, "float32 scan: grid too large");
    hipLaunchKernelGGL(ent->fn, dim3((unsigned)nblocks), dim3(kLanes), 0, st, p);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "scan_fp32_kernel");
}

}  // namespace sfc
