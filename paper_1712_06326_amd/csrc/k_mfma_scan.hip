// Reduced-precision full scan on the matrix cores, with an exact answer.
//
// The full scan (Section I) is split into a filter and an exact refinement
// (the filter-and-refine idea of Fig. 1d applied to the whole dictionary):
//
//   filter: with byte codes x' = x - 128 of targets and patches (Section II's
//     byte quantisation), the quantised masked cost
//         Eq = sum_known (t' - v')^2 = T2 + sum_k A[q,k] B[c,k]
//     is one bf16 GEMM. Per pixel rho the operands hold C + 2 columns:
//         A = [-2 m t'_ch (each channel), 256 m, m]
//         B = [v'_ch (each channel),     s >> 8, s & 255],  s = sum_ch v'^2,
//     so the known part of sum v'^2 costs two columns per pixel instead of
//     two per element. Every operand is an integer of at most 8 significant
//     bits (exact in bf16), every product is exact in float32, and the
//     float32 accumulators are drained into int32 before the sum of the
//     absolute products since the last drain could reach 2^24, so the
//     result is the exact integer whatever the MFMA's summation order.
//   bound: the float cost and Eq differ only by the quantisation residuals
//     (at most 0.5 + 6e-5 per value) and the float32 chain's rounding, so
//       LB(Eq) <= cost <= UB(Eq)
//     with LB/UB from the triangle inequality. Pass 1 records each query's
//     minimum Eq per candidate tile, hence tau = UB(min Eq) >= the optimum;
//     pass 2 revisits only the tiles whose minimum can reach tau and collects
//     every candidate with LB(Eq) <= tau, a set that contains every optimal
//     patch (ties included).
//   refine: the collected candidates are rescored with the exact float32
//     cost; the (cost, id) minimum over them is the full scan's answer.
//   Queries whose set overflows its capacity, or whose target lies outside
//   the quantisation range, are answered by the float32 scan instead.
#include "mfma_scan.hpp"

namespace sfc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}

__device__ inline uint16_t bf16_bits_of_int(int v) {
    // exact for |v| with at most 8 significant bits (all operands here)
    return (uint16_t)(__float_as_uint((float)v) >> 16);
}

// Operands are stored chunk-major: column k of row c at
// ((k / 32) * rows + c) * 32 + k % 32, so the 32-column chunk of a tile's
// rows is one contiguous block.
__device__ inline int64_t blocked_index(int64_t row, int k, int64_t rows) {
    return ((int64_t)(k >> 5) * rows + row) * 32 + (k & 31);
}

// B[c][k] for dictionary entry c (rank order): per pixel C codes v', then
// the high and low byte of sum_ch v'^2; zero rows pad n to the tile size.
// One thread writes 8 consecutive columns of a row (16 bytes); four lanes
// cover a row's 32-column chunk and a wave 16 consecutive rows of it, one
// contiguous kilobyte. blockIdx.y is the chunk.
__global__ __launch_bounds__(256) void dict_operand_kernel(
    const uint8_t* __restrict__ xq, const uint32_t* __restrict__ dict, int64_t n, int64_t npad,
    const int32_t* __restrict__ elem_off, int Kd, int C, int Kp, uint16_t* __restrict__ B) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npad * 4) return;
    const int64_t c = t >> 2;
    const int cols = C + 2;
    const int k0 = (int)blockIdx.y * 32 + (int)(t & 3) * 8;
    int rho = k0 / cols, j = k0 - rho * cols;
    const uint8_t* base = c < n ? xq + (int64_t)dict[c] * C : nullptr;
    uint32_t w[4];
    int sq = -1;   // sum of squares of the current pixel, once its first norm column needs it
    // up to four channels: the pixel's codes are loaded once, in registers
    int px0 = 0, px1 = 0, px2 = 0, px3 = 0, prho = -1;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        int v = 0;
        if (base && rho < Kd && C <= 4) {
            if (rho != prho) {
                const uint8_t* pp = base + elem_off[rho * C];   // channels are contiguous
                px0 = (int)pp[0] - 128;
                px1 = C > 1 ? (int)pp[1] - 128 : 0;
                px2 = C > 2 ? (int)pp[2] - 128 : 0;
                px3 = C > 3 ? (int)pp[3] - 128 : 0;
                sq = px0 * px0 + px1 * px1 + px2 * px2 + px3 * px3;
                prho = rho;
            }
            v = j == 0 ? px0 : j == 1 ? px1 : j == 2 ? px2 : j == 3 ? px3 : 0;
            if (j >= C) v = (j == C) ? (sq >> 8) : (sq & 255);
        } else if (base && rho < Kd) {
            if (j < C) {
                v = (int)base[elem_off[rho * C + j]] - 128;
            } else {
                if (sq < 0) {
                    sq = 0;
                    for (int ch = 0; ch < C; ch++) {
                        const int x = (int)base[elem_off[rho * C + ch]] - 128;
                        sq += x * x;
                    }
                }
                v = (j == C) ? (sq >> 8) : (sq & 255);
            }
        }
        const uint32_t bits = bf16_bits_of_int(v);
        if (e & 1) w[e >> 1] |= bits << 16;
        else w[e >> 1] = bits;
        if (++j == cols) {
            j = 0;
            rho++;
            sq = -1;
        }
    }
    *reinterpret_cast<u32x4*>(B + blocked_index(c, k0, npad)) = u32x4{w[0], w[1], w[2], w[3]};
}

// A[q][k] (same column layout as B), T2[q] = sum_known t'^2, kq[q] = known
// elements, flag[q] = 1 if a known target value lies outside [vmin, vmax]
// (bound not valid).
__global__ void query_operand_kernel(const float* __restrict__ t, const uint8_t* __restrict__ m,
                                     int64_t Q, int64_t Qpad, int Kd, int C, int Kp,
                                     const float* __restrict__ qp,
                                     uint16_t* __restrict__ A, int32_t* __restrict__ T2,
                                     int32_t* __restrict__ kq, int32_t* __restrict__ flag) {
    const int64_t q = blockIdx.x;
    const float vmin = qp[0], s = qp[1], vmax_eff = qp[2];
    const int cols = C + 2;
    int t2 = 0, kn = 0, bad = 0;
    for (int k = threadIdx.x; k < Kp; k += blockDim.x) {
        const int rho = k / cols, j = k - rho * cols;
        int v = 0;
        if (q < Q && rho < Kd && m[q * Kd + rho]) {
            if (j < C) {
                const float x = t[(q * Kd + rho) * C + j];
                float r = __builtin_rintf((x - vmin) * s);
                if (!(r >= 0.0f)) r = 0.0f;
                if (r > 255.0f) r = 255.0f;
                const int tp = (int)r - 128;
                v = -2 * tp;
                t2 += tp * tp;
                kn += 1;
                if (!(x >= vmin && x <= vmax_eff)) bad = 1;
            } else {
                v = (j == C) ? 256 : 1;
            }
        }
        A[blocked_index(q, k, Qpad)] = bf16_bits_of_int(v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        t2 += __shfl_xor(t2, off, 64);
        kn += __shfl_xor(kn, off, 64);
        bad |= __shfl_xor(bad, off, 64);
    }
    __shared__ int s2[4], sk[4], sb[4];
    if ((threadIdx.x & 63) == 0) {
        s2[threadIdx.x >> 6] = t2;
        sk[threadIdx.x >> 6] = kn;
        sb[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0, b = 0, c = 0;
        for (int w = 0; w < (int)blockDim.x / 64; w++) {
            a += s2[w];
            b += sk[w];
            c |= sb[w];
        }
        T2[q] = a;
        kq[q] = b;
        flag[q] = c;
    }
}

// Filter GEMM, persistent: each workgroup walks tiles t = blockIdx.x,
// blockIdx.x + gridDim.x, ... A tile is kFilterRows queries x (64 * TJ)
// candidates, four waves in a 2 x 2 grid, each wave 128 queries x 32*TJ
// candidates as 4 x TJ MFMA 32x32x16 tiles; the accumulators fit two
// workgroups per CU, so one workgroup's loads overlap the other's MFMAs. K is
// staged through LDS in chunks of 32 columns (one contiguous block per
// operand tile in the chunk-major layout), double buffered: the next chunk's
// global loads (the next tile's first chunk during the epilogue) are in
// flight while the current one is multiplied; all of a chunk's fragments
// are requested before its first MFMA. With DRAIN, the float32 accumulators
// are moved into int32 after the chunks flagged in drain_mask.
//   MODE 1: every tile; epilogue = per-query tile minima.
//   MODE 2: the tiles of the work list; epilogue = list candidates <= thr.
//   MODE 3: every tile; epilogue = list candidates <= thr.
// Tile order for modes 1 and 3 (XCD-aware): block b runs on XCD b % 8 (G is
// a multiple of 8, so all its tiles do). The XCDs split the query tiles into
// xq groups and the candidate tiles into 8 / xq bands; each XCD sweeps its
// band candidate tile by candidate tile, all its query tiles per candidate
// tile, so its query operand stays in its L2 and each candidate tile is
// fetched from HBM once per query group.
constexpr int kKC = 32;
constexpr int kLD = kKC + 8;   // bf16 per LDS row (padding against bank conflicts)

__device__ inline bool filter_tile(const FilterArgs& a, int mode, int64_t t, int64_t& qt,
                                   int64_t& ct) {
    if (mode == 2) {
        const uint64_t w = a.work[t];
        qt = (int64_t)(w >> 32);
        ct = (int64_t)(w & 0xffffffffu);
        return true;
    }
    const int x = (int)(t % 8);
    const int64_t slot = t / 8;
    const int ncb = 8 / a.xq, g = x / ncb, bnd = x % ncb;
    const int64_t q_lo = g * a.qtiles / a.xq, q_hi = (g + 1) * a.qtiles / a.xq;
    const int64_t c_lo = bnd * a.ctiles / ncb, c_hi = (bnd + 1) * a.ctiles / ncb;
    const int64_t nq = q_hi - q_lo;
    if (nq <= 0) return false;
    qt = q_lo + slot % nq;
    ct = c_lo + slot / nq;
    return ct < c_hi;
}

// One operand tile's chunk: rows [row0, row0 + 4N*64) of a chunk-major
// operand with `rows` rows, columns [k0, k0 + 32). Thread tid moves 16-byte
// pieces tid + 256 u (row piece / 4, part piece % 4): consecutive threads
// read consecutive bytes.
template <int N>
__device__ __forceinline__ void stage_load(u32x4 (&r)[N], const uint16_t* base, int64_t rows,
                                           int64_t row0, int k0, int tid) {
    const uint16_t* g = base + ((int64_t)(k0 >> 5) * rows + row0) * 32;
#pragma unroll
    for (int u = 0; u < N; u++)
        r[u] = *reinterpret_cast<const u32x4*>(g + (int64_t)(tid + u * 256) * 8);
}

template <int N>
__device__ __forceinline__ void stage_store(const u32x4 (&r)[N], uint16_t* lds, int tid) {
#pragma unroll
    for (int u = 0; u < N; u++) {
        const int e = tid + u * 256, row = e >> 2, part = e & 3;
        *reinterpret_cast<u32x4*>(lds + row * kLD + part * 8) = r[u];
    }
}

__device__ __forceinline__ bf16x8 lds_frag(const uint16_t* p) {
    return *reinterpret_cast<const bf16x8*>(p);
}

template <int MODE, int TJ, bool DRAIN>
__global__ __launch_bounds__(256, 2) void filter_kernel(FilterArgs a) {
    constexpr int TI = 4;
    constexpr int BM = 2 * 32 * TI;   // kFilterRows
    constexpr int BN = 2 * 32 * TJ;
    constexpr int NA = BM * 4 / 256, NB = BN * 4 / 256;   // 16-byte loads per thread
    static_assert(BM == kFilterRows, "query tile");
    // staging buffers [2][BM][kLD] then [2][BN][kLD]; the MODE 1 epilogue
    // reuses them as [4 waves][64 rows][32] int32
    __shared__ __attribute__((aligned(16))) uint16_t smem[2 * BM * kLD + 2 * BN * kLD];
    static_assert(sizeof(smem) >= 4 * 64 * 32 * 4, "epilogue scratch");
    __shared__ int32_t smin[2][BM];
    __shared__ int32_t sth[BM];
    typedef uint16_t TileA[BM][kLD];
    typedef uint16_t TileB[BN][kLD];
    TileA* As = reinterpret_cast<TileA*>(smem);
    TileB* Bs = reinterpret_cast<TileB*>(smem + 2 * BM * kLD);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wq = (wave >> 1) * (32 * TI), wc = (wave & 1) * (32 * TJ);
    const int nk = a.Kp / kKC;
    const int64_t G = gridDim.x;
    const int64_t QR = a.qtiles * BM;     // rows of the query operand
    const int64_t NR = a.crows;           // rows of the dictionary operand
    int64_t t = blockIdx.x, qt = 0, ct = 0;
    while (t < a.ntiles && !filter_tile(a, MODE, t, qt, ct)) t += G;
    if (t >= a.ntiles) return;

    u32x4 ra[NA], rb[NB];
    stage_load<NA>(ra, a.A, QR, qt * BM, 0, tid);
    stage_load<NB>(rb, a.B, NR, ct * BN, 0, tid);
    stage_store<NA>(ra, &As[0][0][0], tid);
    stage_store<NB>(rb, &Bs[0][0][0], tid);
    int p = 0;   // LDS buffer holding the chunk about to be multiplied
    while (true) {
        int64_t nt = t + G, nqt = 0, nct = 0;
        while (nt < a.ntiles && !filter_tile(a, MODE, nt, nqt, nct)) nt += G;
        const bool more = nt < a.ntiles;
        if (MODE != 1) {
            // this tile's query thresholds (read after the next barrier); a
            // query whose list is full takes no more hits: its count is
            // raised above the capacity first, so that the float32 scan
            // answers it even if the count had stopped exactly at the
            // capacity (hits dropped here would otherwise go unnoticed)
            const int64_t q = qt * BM + tid;
            int32_t th = (int32_t)0x80000000;
            if (q < a.Q) {
                const int32_t c = a.cnt[q];
                if (c < a.cap) th = a.thr[q] - a.T2[q];
                else if (c == a.cap) atomicMax(&a.cnt[q], a.cap + 1);
            }
            sth[tid] = th;
        }
        __syncthreads();
        f32x16 acc[TI][TJ];
        int32_t iacc[DRAIN ? TI : 1][DRAIN ? TJ : 1][16];
#pragma unroll
        for (int i = 0; i < TI; i++)
#pragma unroll
            for (int j = 0; j < TJ; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[i][j][r] = 0.0f;
        if (DRAIN) {
#pragma unroll
            for (int i = 0; i < (DRAIN ? TI : 1); i++)
#pragma unroll
                for (int j = 0; j < (DRAIN ? TJ : 1); j++)
#pragma unroll
                    for (int r = 0; r < 16; r++) iacc[i][j][r] = 0;
        }
        for (int kc = 0; kc < nk; kc++) {
            if (kc + 1 < nk) {
                stage_load<NA>(ra, a.A, QR, qt * BM, (kc + 1) * kKC, tid);
                stage_load<NB>(rb, a.B, NR, ct * BN, (kc + 1) * kKC, tid);
            } else if (more) {
                stage_load<NA>(ra, a.A, QR, nqt * BM, 0, tid);
                stage_load<NB>(rb, a.B, NR, nct * BN, 0, tid);
            }
            constexpr int KS = kKC / 16;
            bf16x8 fa[KS][TI], fb[KS][TJ];
#pragma unroll
            for (int k = 0; k < KS; k++) {
                const int kofs = k * 16 + (lane >> 5) * 8;
#pragma unroll
                for (int i = 0; i < TI; i++)
                    fa[k][i] = lds_frag(&As[p][wq + i * 32 + (lane & 31)][kofs]);
#pragma unroll
                for (int j = 0; j < TJ; j++)
                    fb[k][j] = lds_frag(&Bs[p][wc + j * 32 + (lane & 31)][kofs]);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < KS; k++)
#pragma unroll
                for (int i = 0; i < TI; i++)
#pragma unroll
                    for (int j = 0; j < TJ; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[k][i], fb[k][j],
                                                                           acc[i][j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            if (DRAIN && ((a.drain_mask[kc >> 6] >> (kc & 63)) & 1ull)) {
#pragma unroll
                for (int i = 0; i < (DRAIN ? TI : 1); i++)
#pragma unroll
                    for (int j = 0; j < (DRAIN ? TJ : 1); j++)
#pragma unroll
                        for (int r = 0; r < 16; r++) {
                            iacc[i][j][r] += (int32_t)acc[i][j][r];
                            acc[i][j][r] = 0.0f;
                        }
            }
            if (kc + 1 < nk) {
                stage_store<NA>(ra, &As[p ^ 1][0][0], tid);
                stage_store<NB>(rb, &Bs[p ^ 1][0][0], tid);
                __syncthreads();
                p ^= 1;
            }
        }
        // epilogue: lane owns candidate column (lane & 31) of each 32x32 tile
        // and query rows (r/4)*8 + (lane/32)*4 + r%4
        const int64_t q0 = qt * BM, c0 = ct * BN;
        if (MODE == 1) {
            // per query: minimum over the tile's candidates. Each wave
            // reduces its TJ columns per lane, then transposes 64 rows at a
            // time through LDS (the staging buffers, idle once every wave
            // has passed the barrier) and reads one row per lane.
            __syncthreads();
            int32_t* ws = reinterpret_cast<int32_t*>(smem) + wave * 64 * 32;
#pragma unroll
            for (int hf = 0; hf < 2; hf++) {
#pragma unroll
                for (int ii = 0; ii < 2; ii++)
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        const int i = hf * 2 + ii;
                        const int row = ii * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                        int32_t mn = 0x7fffffff;
#pragma unroll
                        for (int j = 0; j < TJ; j++) {
                            int32_t v = (int32_t)acc[i][j][r];
                            if (DRAIN) v += iacc[DRAIN ? i : 0][DRAIN ? j : 0][r];
                            if (c0 + wc + j * 32 + (lane & 31) < a.n) mn = min(mn, v);
                        }
                        ws[row * 32 + (lane & 31)] = mn;
                    }
                __builtin_amdgcn_wave_barrier();
                const u32x4* src = reinterpret_cast<const u32x4*>(ws + lane * 32);
                int32_t mn = 0x7fffffff;
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const u32x4 x = src[k];
                    mn = min(mn, min(min((int32_t)x[0], (int32_t)x[1]), min((int32_t)x[2], (int32_t)x[3])));
                }
                smin[wave & 1][wq + hf * 64 + lane] = mn;
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            const int64_t q = q0 + tid;
            const int32_t v = min(smin[0][tid], smin[1][tid]);
            if (q < a.Q && v != 0x7fffffff) atomicMin(&a.tilemin[q * a.ngroups + ct / a.group], v);
        } else {
            // mark the hits (bit (i*16 + r)*TJ + j), then append them in a
            // rolled loop: hits are rare, and the unrolled part needs no
            // addresses
            uint64_t hit[2] = {0, 0};
            const int64_t cl = a.n - (c0 + wc + (lane & 31));   // columns left for this lane
#pragma unroll
            for (int i = 0; i < TI; i++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    const int row = wq + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                    const int32_t th = sth[row];
#pragma unroll
                    for (int j = 0; j < TJ; j++) {
                        int32_t v = (int32_t)acc[i][j][r];
                        if (DRAIN) v += iacc[DRAIN ? i : 0][DRAIN ? j : 0][r];
                        const int bit = (i * 16 + r) * TJ + j;
                        if (v <= th && j * 32 < cl) hit[bit >> 6] |= 1ull << (bit & 63);
                    }
                }
#pragma unroll
            for (int h = 0; h < 2; h++) {
                uint64_t m = hit[h];
                while (m) {
                    const int bit = h * 64 + __builtin_ctzll(m);
                    m &= m - 1;
                    const int j = bit % TJ, ir = bit / TJ, i = ir >> 4, r = ir & 15;
                    const int row = wq + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                    const int64_t q = q0 + row, c = c0 + wc + j * 32 + (lane & 31);
                    const int32_t slot2 = atomicAdd(&a.cnt[q], 1);
                    if (slot2 < a.cap) a.list[q * a.cap + slot2] = a.dict[c];
                }
            }
            // sth and the staging buffers are rewritten for the next tile
            __syncthreads();
        }
        if (!more) break;
        // the next tile's first chunk into the idle buffer
        stage_store<NA>(ra, &As[p ^ 1][0][0], tid);
        stage_store<NB>(rb, &Bs[p ^ 1][0][0], tid);
        p ^= 1;
        t = nt;
        qt = nqt;
        ct = nct;
    }
}

// Pass-2 work list: (query tile, candidate tile) pairs of every tile group
// in which some query of the tile reaches its threshold. One wave per
// (query tile, group).
__global__ __launch_bounds__(256) void select_kernel(const int32_t* __restrict__ tilemin,
                                                     int64_t ngroups, int group, int64_t ctiles,
                                                     const int32_t* __restrict__ thr,
                                                     const int32_t* __restrict__ T2, int64_t Q,
                                                     int64_t qtiles, uint64_t* __restrict__ work,
                                                     unsigned long long* __restrict__ nwork) {
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= qtiles * ngroups) return;
    const int64_t qt = w / ngroups, g = w - qt * ngroups;
    bool need = false;
    for (int64_t q = qt * kFilterRows + lane; q < min(Q, (qt + 1) * kFilterRows); q += 64)
        if (thr[q] >= 0 && tilemin[q * ngroups + g] <= thr[q] - T2[q]) need = true;
    if (__ballot(need) == 0) return;
    const int64_t c_lo = g * group, c_hi = min(ctiles, c_lo + group);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(nwork, (unsigned long long)(c_hi - c_lo));
    base = __shfl(base, 0, 64);
    for (int64_t c = c_lo + lane; c < c_hi; c += 64)
        work[base + (c - c_lo)] = ((uint64_t)qt << 32) | (uint64_t)c;
}

// Rigorous threshold: Eq_min = T2 + the minimum over the query's tile
// groups, tau = UB(Eq_min), then the largest Eq with LB <= tau.
// UB(E) = (1+er) ((sqrt E + 2 dm sqrt k)/s)^2, LB(E) = (1-er) (max(0, sqrt E -
// 2 dm sqrt k)/s)^2, dm = 0.5 + 6e-5 (residual of a byte code), er = (k+4)
// 2^-23 (float32 chain and difference rounding). Computed in float64 with an
// extra relative margin of 1e-9. One wave per query.
__global__ __launch_bounds__(256) void threshold_kernel(const int32_t* __restrict__ tilemin,
                                                        int64_t ngroups,
                                                        const int32_t* __restrict__ T2,
                                                        const int32_t* __restrict__ kq,
                                                        const int32_t* __restrict__ flag,
                                                        const float* __restrict__ qp, int64_t Q,
                                                        int32_t* __restrict__ thr) {
    const int lane = threadIdx.x & 63;
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (q >= Q) return;
    int32_t mn = 0x7fffffff;
    for (int64_t g = lane; g < ngroups; g += 64) mn = min(mn, tilemin[q * ngroups + g]);
    for (int off = 32; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off, 64));
    if (lane != 0) return;
    const double s = (double)qp[1];
    const double k = (double)kq[q];
    const double er = (k + 4.0) * 0x1p-23;
    const double slack = 2.0 * (0.5 + 6e-5) * sqrt(k);
    if (s <= 0.0 || flag[q] || mn == 0x7fffffff) {
        thr[q] = -1;   // force the float32 scan
        return;
    }
    const double eqmin = (double)T2[q] + (double)mn;
    const double ub = (1.0 + er) * ((sqrt(eqmin) + slack) / s) * ((sqrt(eqmin) + slack) / s) *
                      (1.0 + 1e-9);
    const double root = slack + s * sqrt(ub / (1.0 - er)) * (1.0 + 1e-9);
    const double e = floor(root * root) + 1.0;
    thr[q] = e > 2.0e9 ? 2000000000 : (int32_t)e;
}

// Threshold from a known upper bound tau on the optimum (the exact cost of
// some candidate): every candidate whose cost can be <= tau has
// LB(Eq) <= tau, i.e. sqrt Eq <= 2 dm sqrt k + s sqrt(tau / (1 - er)).
__global__ void seed_threshold_kernel(const float* __restrict__ tau, const int32_t* __restrict__ kq,
                                      const int32_t* __restrict__ flag, const float* __restrict__ qp,
                                      int64_t Q, int32_t* __restrict__ thr) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const double s = (double)qp[1];
    const double k = (double)kq[q];
    const double er = (k + 4.0) * 0x1p-23;
    const double slack = 2.0 * (0.5 + 6e-5) * sqrt(k);
    const double tq = (double)tau[q];
    if (s <= 0.0 || flag[q] || !(tq >= 0.0 && tq < 1e30)) {
        thr[q] = -1;   // force the float32 scan
        return;
    }
    const double root = slack + s * sqrt(tq / (1.0 - er)) * (1.0 + 1e-9);
    const double e = floor(root * root) + 1.0;
    thr[q] = e > 2.0e9 ? 2000000000 : (int32_t)e;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

// Largest |product| a column of the operands can contribute.
int64_t column_bound(int k, int Kd, int C) {
    const int rho = k / (C + 2), j = k % (C + 2);
    if (rho >= Kd) return 0;
    if (j < C) return 32768;            // |-2 t' v'| <= 2 * 128 * 128
    if (j == C) return 16384LL * C;     // 256 * (s >> 8) <= s <= C * 128^2
    return 255;                         // s & 255
}

}  // namespace

int64_t mfma_kp(int Kd, int C) { return (((int64_t)Kd * (C + 2) + kKC - 1) / kKC) * kKC; }

sfc_status plan_filter(int Kd, int C, int64_t Q, int64_t n, FilterArgs* a) {
    a->Kp = (int)mfma_kp(Kd, C);
    const int nk = a->Kp / kKC;
    if (nk > 128) return fail(SFC_EUNSUPPORTED, "reduced-precision scan: operand wider than 4096");
    constexpr int64_t kLimit = (1 << 24) - 1;
    int64_t total = 0;
    for (int k = 0; k < a->Kp; k++) total += column_bound(k, Kd, C);
    a->drain_mask[0] = a->drain_mask[1] = 0;
    a->drain = total > kLimit;
    if (a->drain) {
        int64_t run = 0;
        for (int kc = 0; kc < nk; kc++) {
            int64_t cb = 0;
            for (int k = kc * kKC; k < (kc + 1) * kKC; k++) cb += column_bound(k, Kd, C);
            if (run + cb > kLimit) {
                a->drain_mask[(kc - 1) >> 6] |= 1ull << ((kc - 1) & 63);
                run = 0;
            }
            run += cb;
        }
    }
    a->bn = a->drain ? 64 : 128;
    a->Q = Q;
    a->n = n;
    a->ctiles = (n + a->bn - 1) / a->bn;
    a->crows = (n + 255) / 256 * 256;   // the dictionary operand's row count
    a->qtiles = (Q + kFilterRows - 1) / kFilterRows;
    a->ctiles_per_xcd = (a->ctiles + 7) / 8;
    // query groups across the XCDs: the smallest power of two that keeps an
    // XCD's share of the query operand within 2 MiB of its L2
    const int64_t qbytes = (int64_t)kFilterRows * a->Kp * 2;
    a->xq = 1;
    while (a->xq < 8 && ((a->qtiles + a->xq - 1) / a->xq) * qbytes > (int64_t(2) << 20)) a->xq *= 2;
    if (a->xq > a->qtiles) {
        a->xq = 1;
        while (a->xq * 2 <= a->qtiles && a->xq < 8) a->xq *= 2;
    }
    {
        const int ncb = 8 / a->xq;
        int64_t most = 0;
        for (int x = 0; x < 8; x++) {
            const int g = x / ncb, bnd = x % ncb;
            const int64_t nq = (g + 1) * a->qtiles / a->xq - g * a->qtiles / a->xq;
            const int64_t nc = (bnd + 1) * a->ctiles / ncb - bnd * a->ctiles / ncb;
            most = std::max(most, nq * nc);
        }
        a->all_tiles = 8 * most;
    }
    // tile minima kept per group of candidate tiles, at most 64 Mi entries
    const int64_t budget = int64_t(64) << 20;
    int64_t group = (Q * a->ctiles + budget - 1) / budget;
    if (group < 1) group = 1;
    a->group = (int)group;
    a->ngroups = (a->ctiles + group - 1) / group;
    return SFC_OK;
}

sfc_status launch_dict_operand(const uint8_t* xq, const uint32_t* dict, int64_t n, int64_t npad,
                               const int32_t* elem_off, int Kd, int C, int Kp, uint16_t* B,
                               hipStream_t st) {
    if (Kp % 32 != 0 || Kp / 32 > 65535 || npad * 4 > (int64_t)0x7fffffff * 256)
        return fail(SFC_EUNSUPPORTED, "dictionary operand: shape out of range");
    dict_operand_kernel<<<dim3(blocks_for(npad * 4), Kp / 32), 256, 0, st>>>(xq, dict, n, npad,
                                                                             elem_off, Kd, C, Kp, B);
    return launched("dict_operand_kernel");
}

sfc_status launch_query_operand(const float* t, const uint8_t* m, int64_t Q, int64_t Qpad, int Kd,
                                int C, int Kp, const float* qp, uint16_t* A, int32_t* T2,
                                int32_t* kq, int32_t* flag, hipStream_t st) {
    query_operand_kernel<<<(unsigned)Qpad, 256, 0, st>>>(t, m, Q, Qpad, Kd, C, Kp, qp, A, T2, kq,
                                                         flag);
    return launched("query_operand_kernel");
}

namespace {

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

// persistent grid: two workgroups per CU (what the kernel's registers and
// LDS allow), a multiple of 8 so every workgroup stays on one XCD
unsigned persistent_grid(int64_t tiles) {
    int64_t g = std::min<int64_t>(tiles, 2 * (int64_t)device_cus());
    g = (g + 7) / 8 * 8;
    return (unsigned)std::max<int64_t>(8, g);
}

}  // namespace

sfc_status launch_filter_minima(FilterArgs a, hipStream_t st) {
    const int64_t entries = a.Q * a.ngroups;
    fill_i32_kernel<<<(unsigned)std::min<int64_t>(4096, (entries + 255) / 256), 256, 0, st>>>(
        a.tilemin, entries, 0x7fffffff);
    SFC_TRY(launched("fill_i32_kernel"));
    a.ntiles = a.all_tiles;
    const unsigned g = persistent_grid(a.ntiles);
    if (a.drain)
        filter_kernel<1, 1, true><<<g, 256, 0, st>>>(a);
    else
        filter_kernel<1, 2, false><<<g, 256, 0, st>>>(a);
    return launched("filter_kernel");
}

sfc_status launch_filter_list(FilterArgs a, int64_t nwork, hipStream_t st) {
    fill_i32_kernel<<<(unsigned)std::min<int64_t>(4096, (a.Q + 255) / 256), 256, 0, st>>>(
        a.cnt, a.Q, 0);
    SFC_TRY(launched("fill_i32_kernel"));
    if (nwork == 0) return SFC_OK;
    if (nwork > 0) {
        a.ntiles = nwork;
        const unsigned g = persistent_grid(nwork);
        if (a.drain)
            filter_kernel<2, 1, true><<<g, 256, 0, st>>>(a);
        else
            filter_kernel<2, 2, false><<<g, 256, 0, st>>>(a);
    } else {
        a.ntiles = a.all_tiles;
        const unsigned g = persistent_grid(a.ntiles);
        if (a.drain)
            filter_kernel<3, 1, true><<<g, 256, 0, st>>>(a);
        else
            filter_kernel<3, 2, false><<<g, 256, 0, st>>>(a);
    }
    return launched("filter_kernel");
}

sfc_status launch_threshold(const FilterArgs& a, const int32_t* kq, const int32_t* flag,
                            const float* qp, int32_t* thr, hipStream_t st) {
    threshold_kernel<<<blocks_for(a.Q * 64), 256, 0, st>>>(a.tilemin, a.ngroups, a.T2, kq, flag, qp,
                                                           a.Q, thr);
    return launched("threshold_kernel");
}

sfc_status launch_seed_threshold(const float* tau, const int32_t* kq, const int32_t* flag,
                                 const float* qp, int64_t Q, int32_t* thr, hipStream_t st) {
    seed_threshold_kernel<<<blocks_for(Q), 256, 0, st>>>(tau, kq, flag, qp, Q, thr);
    return launched("seed_threshold_kernel");
}

sfc_status launch_select(const FilterArgs& a, uint64_t* work, unsigned long long* nwork,
                         hipStream_t st) {
    zero_u64_kernel<<<1, 1, 0, st>>>(nwork);
    SFC_TRY(launched("zero_u64_kernel"));
    select_kernel<<<blocks_for(a.qtiles * a.ngroups * 64), 256, 0, st>>>(
        a.tilemin, a.ngroups, a.group, a.ctiles, a.thr, a.T2, a.Q, a.qtiles, work, nwork);
    return launched("select_kernel");
}

}  // namespace sfc
