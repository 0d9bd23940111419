// Reduced-precision full scan on the matrix cores, with an exact answer.
//
// The full scan (Section I) is split into a filter and an exact refinement
// (the filter-and-refine idea of Fig. 1d applied to the whole dictionary):
//
//   filter: with byte codes x' = x - 128 of targets and patches (Section II's
//     byte quantisation), the quantised masked cost
//         Eq = sum_known (t' - v')^2 = T2 + sum_e A[q,e] B[c,e]
//     with A = [-2 m t', 128 m, m] and B = [v', v'^2 >> 7, v'^2 & 127]
//     per element is one bf16 GEMM. Every operand is an integer of at most
//     8 significant bits (exact in bf16), every product is exact in float32
//     and every partial sum over at most 340 elements stays below 2^24, so
//     the MFMA result is the exact integer whatever its summation order.
//   bound: the float cost and Eq differ only by the quantisation residuals
//     (at most 0.5 + 6e-5 per value) and the float32 chain's rounding, so
//       LB(Eq) <= cost <= UB(Eq)
//     with LB/UB from the triangle inequality. Pass 1 takes each query's
//     minimum Eq, hence tau = UB(min Eq) >= the optimum; pass 2 collects
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

// B[c][3e + j] for dictionary entry c (rank order), element e.
__global__ void dict_operand_kernel(const uint8_t* __restrict__ xq, const uint32_t* __restrict__ dict,
                                    int64_t n, const int32_t* __restrict__ elem_off, int P, int C,
                                    int Kp, uint16_t* __restrict__ B) {
    const int64_t npad = (n + kMfmaTile - 1) / kMfmaTile * kMfmaTile;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad * Kp;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / Kp;
        const int k = (int)(i - c * Kp);
        const int e = k / 3, j = k - 3 * e;
        int v = 0;
        if (c < n && e < P) {
            const int x = (int)xq[(int64_t)dict[c] * C + elem_off[e]] - 128;
            const int sq = x * x;
            v = (j == 0) ? x : (j == 1 ? (sq >> 7) : (sq & 127));
        }
        B[i] = bf16_bits_of_int(v);
    }
}

// A[q][3e + j], T2[q] = sum_known t'^2, kq[q] = known elements, flag[q] = 1
// if a known target value lies outside [vmin, vmax] (bound not valid).
__global__ void query_operand_kernel(const float* __restrict__ t, const uint8_t* __restrict__ m,
                                     int64_t Q, int Kd, int C, int Kp, const float* __restrict__ qp,
                                     uint16_t* __restrict__ A, int32_t* __restrict__ T2,
                                     int32_t* __restrict__ kq, int32_t* __restrict__ flag) {
    const int64_t q = blockIdx.x;
    const float vmin = qp[0], s = qp[1], vmax_eff = qp[2];
    int t2 = 0, kn = 0, bad = 0;
    for (int k = threadIdx.x; k < Kp; k += blockDim.x) {
        const int e = k / 3, j = k - 3 * e;
        int v = 0;
        if (q < Q && e < Kd * C && m[q * Kd + e / C]) {
            const float x = t[q * Kd * C + e];
            float r = __builtin_rintf((x - vmin) * s);
            if (!(r >= 0.0f)) r = 0.0f;
            if (r > 255.0f) r = 255.0f;
            const int tp = (int)r - 128;
            v = (j == 0) ? -2 * tp : (j == 1 ? 128 : 1);
            if (j == 0) {
                t2 += tp * tp;
                kn += 1;
                if (!(x >= vmin && x <= vmax_eff)) bad = 1;
            }
        }
        A[q * Kp + k] = bf16_bits_of_int(v);
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

// One workgroup: a 128-query x 128-candidate tile; four waves of 64 x 64,
// each 2 x 2 MFMA 32x32x16 tiles, operands staged through LDS in K-chunks of
// 32. The float32 accumulators are drained into integers every kDrainK
// elements of K so no partial sum reaches 2^24.
template <int PASS>
__global__ __launch_bounds__(256) void filter_kernel(FilterArgs a) {
    constexpr int KC = 32;
    constexpr int LDA = KC + 8;   // bf16 elements per LDS row (padding against conflicts)
    __shared__ uint16_t As[kMfmaTile][LDA];
    __shared__ uint16_t Bs[kMfmaTile][LDA];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // XCD-aware order: blocks with the same candidate tile run on one XCD
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % 8, slot = b / 8;
    const int64_t ct = xcd * a.ctiles_per_xcd + slot % a.ctiles_per_xcd;
    const int64_t qt = slot / a.ctiles_per_xcd;
    if (ct >= a.ctiles || qt >= a.qtiles) return;
    const int64_t q0 = qt * kMfmaTile, c0 = ct * kMfmaTile;
    const int wq = (wave >> 1) * 64, wc = (wave & 1) * 64;

    f32x16 acc[2][2];
    int32_t iacc[2][2][16];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                acc[i][j][r] = 0.0f;
                iacc[i][j][r] = 0;
            }
    const uint16_t* Ag = a.A + q0 * a.Kp;
    const uint16_t* Bg = a.B + c0 * a.Kp;
    int since_drain = 0;
    for (int k0 = 0; k0 < a.Kp; k0 += KC) {
        // stage: 128 rows x 32 bf16 = 8 KB per operand; 16 bytes per thread each
        {
            const int r = tid >> 1, h = (tid & 1) * 16;
            const uint4* ga = reinterpret_cast<const uint4*>(Ag + (int64_t)r * a.Kp + k0 + h);
            const uint4* gb = reinterpret_cast<const uint4*>(Bg + (int64_t)r * a.Kp + k0 + h);
            const uint4 va0 = ga[0], va1 = ga[1], vb0 = gb[0], vb1 = gb[1];
            __syncthreads();
            *reinterpret_cast<uint4*>(&As[r][h]) = va0;
            *reinterpret_cast<uint4*>(&As[r][h + 8]) = va1;
            *reinterpret_cast<uint4*>(&Bs[r][h]) = vb0;
            *reinterpret_cast<uint4*>(&Bs[r][h + 8]) = vb1;
            __syncthreads();
        }
#pragma unroll
        for (int kk = 0; kk < KC; kk += 16) {
            const int kofs = kk + (lane >> 5) * 8;
            bf16x8 fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; i++) {
                union { uint4 u; bf16x8 v; } ua, ub;
                ua.u = *reinterpret_cast<const uint4*>(&As[wq + i * 32 + (lane & 31)][kofs]);
                ub.u = *reinterpret_cast<const uint4*>(&Bs[wc + i * 32 + (lane & 31)][kofs]);
                fa[i] = ua.v;
                fb[i] = ub.v;
            }
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        since_drain += KC;
        if (since_drain >= kDrainK) {
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        iacc[i][j][r] += (int32_t)acc[i][j][r];
                        acc[i][j][r] = 0.0f;
                    }
            since_drain = 0;
        }
    }
    // epilogue: lane owns candidate column (lane & 31) of each 32x32 tile and
    // query rows (r/4)*8 + (lane/32)*4 + r%4
    if (PASS == 1) {
        // per query row: minimum over the wave's 64 candidates, one atomic
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int64_t q = q0 + wq + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                int32_t mn = 0x7fffffff;
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int64_t c = c0 + wc + j * 32 + (lane & 31);
                    const int32_t eq = a.T2[q] + iacc[i][j][r] + (int32_t)acc[i][j][r];
                    if (c < a.n) mn = min(mn, eq);
                }
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off, 64));
                if ((lane & 31) == 0 && q < a.Q && mn != 0x7fffffff) atomicMin(&a.eqmin[q], mn);
            }
    } else {
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int64_t q = q0 + wq + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                if (q >= a.Q) continue;
                const int32_t th = a.thr[q] - a.T2[q];
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int64_t c = c0 + wc + j * 32 + (lane & 31);
                    const int32_t part = iacc[i][j][r] + (int32_t)acc[i][j][r];
                    if (c < a.n && part <= th) {
                        const int32_t slot2 = atomicAdd(&a.cnt[q], 1);
                        if (slot2 < a.cap) a.list[q * a.cap + slot2] = a.dict[c];
                    }
                }
            }
    }
}

// Rigorous threshold: tau = UB(Eq_min), then the largest Eq with LB <= tau.
// UB(E) = (1+er) ((sqrt E + 2 dm sqrt k)/s)^2, LB(E) = (1-er) (max(0, sqrt E -
// 2 dm sqrt k)/s)^2, dm = 0.5 + 6e-5 (residual of a byte code), er = (k+4)
// 2^-23 (float32 chain and difference rounding). Computed in float64 with an
// extra relative margin of 1e-9.
__global__ void threshold_kernel(const int32_t* __restrict__ eqmin, const int32_t* __restrict__ kq,
                                 const int32_t* __restrict__ flag, const float* __restrict__ qp,
                                 int64_t Q, int32_t* __restrict__ thr) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const double s = (double)qp[1];
    const double k = (double)kq[q];
    const double er = (k + 4.0) * 0x1p-23;
    const double slack = 2.0 * (0.5 + 6e-5) * sqrt(k);
    if (s <= 0.0 || flag[q] || eqmin[q] == 0x7fffffff) {
        thr[q] = -1;   // force the float32 scan
        return;
    }
    const double ub = (1.0 + er) * ((sqrt((double)eqmin[q]) + slack) / s) *
                      ((sqrt((double)eqmin[q]) + slack) / s) * (1.0 + 1e-9);
    const double root = slack + s * sqrt(ub / (1.0 - er)) * (1.0 + 1e-9);
    const double e = floor(root * root) + 1.0;
    thr[q] = e > 2.0e9 ? 2000000000 : (int32_t)e;
}

__global__ void init_filter_kernel(int32_t* eqmin, int32_t* cnt, int64_t Q) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < Q) {
        eqmin[q] = 0x7fffffff;
        cnt[q] = 0;
    }
}

}  // namespace

int64_t mfma_kp(int P) { return ((3 * (int64_t)P + 31) / 32) * 32; }

sfc_status launch_dict_operand(const uint8_t* xq, const uint32_t* dict, int64_t n,
                               const int32_t* elem_off, int P, int C, uint16_t* B, hipStream_t st) {
    const int64_t Kp = mfma_kp(P);
    const int64_t npad = (n + kMfmaTile - 1) / kMfmaTile * kMfmaTile;
    const unsigned nb = (unsigned)std::min<int64_t>(1 << 20, (npad * Kp + 255) / 256);
    dict_operand_kernel<<<nb, 256, 0, st>>>(xq, dict, n, elem_off, P, C, (int)Kp, B);
    return launched("dict_operand_kernel");
}

sfc_status launch_query_operand(const float* t, const uint8_t* m, int64_t Q, int64_t Qpad, int Kd,
                                int C, const float* qp, uint16_t* A, int32_t* T2, int32_t* kq,
                                int32_t* flag, hipStream_t st) {
    const int Kp = (int)mfma_kp(Kd * C);
    query_operand_kernel<<<(unsigned)Qpad, 256, 0, st>>>(t, m, Q, Kd, C, Kp, qp, A, T2, kq, flag);
    return launched("query_operand_kernel");
}

sfc_status launch_filter(FilterArgs a, int pass, hipStream_t st) {
    a.ctiles = (a.n + kMfmaTile - 1) / kMfmaTile;
    a.qtiles = (a.Q + kMfmaTile - 1) / kMfmaTile;
    a.ctiles_per_xcd = (a.ctiles + 7) / 8;
    const int64_t nb = 8 * a.ctiles_per_xcd * a.qtiles;
    if (nb > 0x7fffffff) return fail(SFC_EUNSUPPORTED, "reduced-precision scan grid too large");
    if (pass == 1) {
        init_filter_kernel<<<blocks_for(a.Q), 256, 0, st>>>(a.eqmin, a.cnt, a.Q);
        SFC_TRY(launched("init_filter_kernel"));
        filter_kernel<1><<<(unsigned)nb, 256, 0, st>>>(a);
    } else {
        filter_kernel<2><<<(unsigned)nb, 256, 0, st>>>(a);
    }
    return launched("filter_kernel");
}

sfc_status launch_threshold(const int32_t* eqmin, const int32_t* kq, const int32_t* flag,
                            const float* qp, int64_t Q, int32_t* thr, hipStream_t st) {
    threshold_kernel<<<blocks_for(Q), 256, 0, st>>>(eqmin, kq, flag, qp, Q, thr);
    return launched("threshold_kernel");
}

}  // namespace sfc
