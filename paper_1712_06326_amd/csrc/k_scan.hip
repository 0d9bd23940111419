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
constexpr int kScanQB = 16;

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
};

// Lane-level running best over the tiles of a workgroup: candidates of later
// tiles have larger ids, so a strict comparison keeps the lowest id on ties.
template <int ND, int K, int C, int QB>
__global__ __launch_bounds__(kLanes) void scan_fp32_kernel(ScanParams p) {
    constexpr int H = (K - 1) / 2;
    constexpr int ROWS = (ND == 2) ? K : K * K;
    constexpr int TW = kLanes + K - 1;
    constexpr int RW = K * C;
    constexpr int TILE = ROWS * TW * C;
    extern __shared__ float smem[];
    float* tile = smem;
    uint32_t* sred = reinterpret_cast<uint32_t*>(smem + TILE);  // [4 waves][QB][2]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.y * p.q_per_wg;
    const int64_t q1 = min(p.Q, q0 + p.q_per_wg);
    if (q0 >= q1) return;
    const int64_t tl0 = (int64_t)blockIdx.x * p.tiles_per_wg;
    const int64_t tl1 = min(p.n_tiles, tl0 + p.tiles_per_wg);

    for (int64_t qb = q0; qb < q1; qb += QB) {
        uint32_t bcost[QB], bid[QB];
#pragma unroll
        for (int qi = 0; qi < QB; qi++) {
            bcost[qi] = 0xffffffffu;
            bid[qi] = 0xffffffffu;
        }
        for (int64_t tl = tl0; tl < tl1; tl++) {
            const int64_t line = tl / p.tiles_per_line;
            const int64_t x0 = (tl - line * p.tiles_per_line) * kLanes;
            int64_t base;
            if (ND == 2) {
                base = (line + H) * p.stride[0];
            } else {
                const int64_t iy = p.shape[1] - 2 * H;
                const int64_t z = line / iy, y = line - z * iy;
                base = (z + H) * p.stride[0] + (y + H) * p.stride[1];
            }
            __syncthreads();
            for (int i = tid; i < TILE; i += kLanes) {
                const int r = i / (TW * C);
                const int rem = i - r * TW * C;
                const int j = rem / C;
                const int ch = rem - j * C;
                const int64_t xv = x0 + j;
                float val = 0.0f;
                if (xv < p.shape[ND - 1]) {
                    int64_t roff;
                    if (ND == 2) roff = (int64_t)(r - H) * p.stride[0];
                    else roff = (int64_t)(r / K - H) * p.stride[0] + (int64_t)(r % K - H) * p.stride[1];
                    val = p.vol[(base + roff + xv) * C + ch];
                }
                tile[i] = val;
            }
            __syncthreads();
            const int64_t xi = x0 + tid;
            const bool cvalid = (xi < p.line_len) && p.valid[base + xi + H];
            const uint32_t cid = (uint32_t)(base + xi + H);

            float acc[QB];
#pragma unroll
            for (int qi = 0; qi < QB; qi++) acc[qi] = 0.0f;
            for (int r = 0; r < ROWS; r++) {
                // masks of the QB queries for row r are contiguous (row-major [rows][Qpad])
                const uint32_t* mrb = p.rowmask + (int64_t)r * p.qpad + qb;
                uint32_t mrow[QB];
                uint32_t orm = 0;
#pragma unroll
                for (int qi = 0; qi < QB; qi++) {
                    mrow[qi] = ldu(mrb + qi);
                    orm |= mrow[qi];
                }
                if (orm == 0) continue;
                float v[RW];
                const float* trow = tile + (r * TW + tid) * C;
#pragma unroll
                for (int i = 0; i < RW; i++) v[i] = trow[i];
                const float* tb = p.t + (qb * ROWS + r) * RW;
#pragma unroll
                for (int qi = 0; qi < QB; qi++) {
                    const uint32_t mr = mrow[qi];
                    if (mr == 0) continue;
                    float tr[RW];
#pragma unroll
                    for (int i = 0; i < RW; i++) tr[i] = ldu(tb + qi * ROWS * RW + i);
#pragma unroll
                    for (int dx = 0; dx < K; dx++) {
                        if (mr & (1u << dx)) {
#pragma unroll
                            for (int ch = 0; ch < C; ch++) {
                                const float d = tr[dx * C + ch] - v[dx * C + ch];
                                acc[qi] = __builtin_fmaf(d, d, acc[qi]);
                            }
                        }
                    }
                }
            }
            if (cvalid) {
#pragma unroll
                for (int qi = 0; qi < QB; qi++) {
                    const uint32_t cb = __float_as_uint(acc[qi]);
                    if (cb < bcost[qi]) {
                        bcost[qi] = cb;
                        bid[qi] = cid;
                    }
                }
            }
        }
        // (cost, id) minimum over the workgroup, then one global atomic per query
#pragma unroll
        for (int qi = 0; qi < QB; qi++) {
            uint32_t c = bcost[qi];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) c = min(c, (uint32_t)__shfl_xor((int)c, off, 64));
            const uint64_t bal = __ballot(bcost[qi] == c);
            const int first = __ffsll((unsigned long long)bal) - 1;
            const uint32_t id = (uint32_t)__shfl((int)bid[qi], first, 64);
            if (lane == 0) {
                sred[(wave * QB + qi) * 2] = c;
                sred[(wave * QB + qi) * 2 + 1] = id;
            }
        }
        __syncthreads();
        if (tid < QB && qb + tid < q1) {
            uint64_t best = ~0ull;
            for (int w = 0; w < kLanes / 64; w++) {
                const uint32_t c = sred[(w * QB + tid) * 2], id = sred[(w * QB + tid) * 2 + 1];
                if (c != 0xffffffffu) {
                    const uint64_t pk = ((uint64_t)c << 32) | id;
                    if (pk < best) best = pk;
                }
            }
            if (best != ~0ull)
                atomicMin((unsigned long long*)&p.best[qb + tid], (unsigned long long)best);
        }
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

template <int ND, int K, int C>
constexpr int scan_qb() {
    return kScanQB;
}

template <int ND, int K, int C>
ScanFn pick() {
    return scan_fp32_kernel<ND, K, C, scan_qb<ND, K, C>()>;
}

struct ScanEntry {
    int nd, K, C;
    ScanFn fn;
    int qb;
};

#define SFC_SCAN_ENTRY(ND, K, C) {ND, K, C, pick<ND, K, C>(), scan_qb<ND, K, C>()}

const ScanEntry kScanTable[] = {
    SFC_SCAN_ENTRY(2, 3, 1), SFC_SCAN_ENTRY(2, 3, 2), SFC_SCAN_ENTRY(2, 3, 3),
    SFC_SCAN_ENTRY(2, 5, 1), SFC_SCAN_ENTRY(2, 5, 2), SFC_SCAN_ENTRY(2, 5, 3),
    SFC_SCAN_ENTRY(2, 7, 1), SFC_SCAN_ENTRY(2, 7, 2), SFC_SCAN_ENTRY(2, 7, 3),
    SFC_SCAN_ENTRY(2, 9, 1), SFC_SCAN_ENTRY(2, 9, 2), SFC_SCAN_ENTRY(2, 9, 3),
    SFC_SCAN_ENTRY(2, 11, 1), SFC_SCAN_ENTRY(2, 11, 3),
    SFC_SCAN_ENTRY(2, 13, 1), SFC_SCAN_ENTRY(2, 13, 3),
    SFC_SCAN_ENTRY(3, 3, 1), SFC_SCAN_ENTRY(3, 3, 2),
    SFC_SCAN_ENTRY(3, 5, 1), SFC_SCAN_ENTRY(3, 5, 2),
    SFC_SCAN_ENTRY(3, 7, 1),
};

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

bool scan_supported(int nd, int K, int C) {
    for (const auto& e : kScanTable)
        if (e.nd == nd && e.K == K && e.C == C) return true;
    return false;
}

int64_t scan_qpad(int64_t Q) { return ((Q + kScanQB - 1) / kScanQB) * kScanQB; }

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
    const ScanEntry* ent = nullptr;
    for (const auto& e : kScanTable)
        if (e.nd == g.nd && e.K == g.K && e.C == g.C) ent = &e;
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
    p.tiles_per_line = (p.line_len + kLanes - 1) / kLanes;
    p.n_tiles = n_lines * p.tiles_per_line;
    // queries per workgroup (LDS holds one 8-byte best per query)
    int64_t qpw = a.query_block > 0 ? a.query_block : 1024;
    qpw = ((qpw + ent->qb - 1) / ent->qb) * ent->qb;
    if (qpw > a.Q) qpw = ((a.Q + ent->qb - 1) / ent->qb) * ent->qb;
    p.q_per_wg = qpw;
    p.qpad = scan_qpad(a.Q);
    const int64_t qsplit = (a.Q + qpw - 1) / qpw;
    int64_t tpw = (p.n_tiles * qsplit + 2047) / 2048;
    if (tpw < 1) tpw = 1;
    p.tiles_per_wg = tpw;
    const int64_t chunks = (p.n_tiles + tpw - 1) / tpw;
    const int rows = g.rows;
    const size_t tile_floats = (size_t)rows * (kLanes + g.K - 1) * g.C;
    const size_t lds = tile_floats * sizeof(float) + (size_t)(kLanes / 64) * ent->qb * 8;
    if (lds > 160 * 1024)
        return fail(SFC_EUNSUPPORTED, "float32 scan: LDS tile too large");
    if (qsplit > 65535) return fail(SFC_EUNSUPPORTED, "float32 scan: too many queries");
    dim3 grid((unsigned)chunks, (unsigned)qsplit);
    if (lds > 64 * 1024) {
        hipError_t ea = hipFuncSetAttribute((const void*)ent->fn,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (ea != hipSuccess) return check_hip(ea, "scan_fp32_kernel LDS attribute");
    }
    hipLaunchKernelGGL(ent->fn, grid, dim3(kLanes), lds, st, p);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "scan_fp32_kernel");
}

}  // namespace sfc
