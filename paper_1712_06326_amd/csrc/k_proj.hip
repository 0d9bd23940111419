// Index build, part 2 (Sections II.A-C): principal coordinates of every
// dictionary patch by an MFMA GEMM, their grid cells on the shifted curves
// and the curve keys.
//
// Projection: Y[n, S*D] = X[n, P] * Wcat[P, S*D], where row c of X is the
// byte-coded patch of dictionary entry c (an implicit im2col gathered from
// the quantised volume into LDS) and Wcat holds every subset's int8 basis in
// its own D columns (zero outside the subset's elements). The GEMM runs on
// v_mfma_i32_32x32x32_i8 over (x - 128) (a byte XOR 0x80 is that value as
// int8) and adds 128 * (column sum of W) afterwards: integer arithmetic
// throughout, so the coordinates are exact for any patch size.
#include "build.hpp"
#include "keys.hpp"
#include "proj.hpp"

namespace sfc {

namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}

constexpr int kProjRows = 128;   // patches per workgroup (32 per wave)

template <int NT>
__global__ __launch_bounds__(256) void proj_kernel(ProjArgs a) {
    extern __shared__ __align__(16) uint8_t As[];   // [kProjRows][Pk + 16]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int stride = a.Pk + 16;
    const int64_t base = (int64_t)blockIdx.x * kProjRows;
    // gather by runs: a patch is P / run runs of `run` contiguous bytes
    const int nruns = a.P / a.run;
    for (int i = tid; i < kProjRows * nruns; i += 256) {
        const int r = i / nruns, j = i - r * nruns;
        const int64_t c = base + r;
        if (c >= a.cnt) continue;
        const uint8_t* src = a.xq + (int64_t)a.dict[a.r0 + c] * a.C + a.elem_off[j * a.run];
        uint8_t* dst = As + r * stride + j * a.run;
        for (int e = 0; e < a.run; e++) dst[e] = src[e];
    }
    // the padding elements meet zero weights; cleared so no stale bytes enter
    const int npad = a.Pk - a.P;
    for (int i = tid; i < kProjRows * npad; i += 256) {
        const int r = i / npad;
        As[r * stride + a.P + (i - r * npad)] = 0;
    }
    __syncthreads();
    i32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int i = 0; i < 16; i++) acc[t][i] = 0;
    const int row = wave * 32 + (lane & 31);
    // each half-wave supplies 16 of the 32 depth positions of a step, the
    // same positions for the patch row and the weight column
    const int kh = (lane >> 5) * 16;
    const bool live = base + wave * 32 < a.cnt;
    if (live) {
        for (int k0 = 0; k0 < a.Pk; k0 += 32) {
            i32x4 A = *reinterpret_cast<const i32x4*>(As + row * stride + k0 + kh);
#pragma unroll
            for (int v = 0; v < 4; v++) A[v] ^= (int)0x80808080u;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int8_t* bp = a.Wt + (int64_t)(t * 32 + (lane & 31)) * a.Pk + k0 + kh;
                const i32x4 B = *reinterpret_cast<const i32x4*>(bp);
                acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B, acc[t], 0, 0, 0);
            }
        }
    }
    // epilogue: lane holds column (lane & 31) of each tile, rows
    // (i/4)*8 + (lane/32)*4 + i%4 of the wave's 32 patches.
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int col = t * 32 + (lane & 31);
        const int ws = a.wsum[col];
        int mn = 0x7fffffff, mx = (int)0x80000000;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const int r = (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
            const int64_t c = base + wave * 32 + r;
            const int yv = acc[t][i] + ws;
            if (c < a.cnt && col < a.ncols) {
                if (a.y) a.y[c * a.ystride + col] = yv;
                mn = min(mn, yv);
                mx = max(mx, yv);
            }
        }
        mn = min(mn, __shfl_xor(mn, 32, 64));
        mx = max(mx, __shfl_xor(mx, 32, 64));
        if (lane < 32 && col < a.ncols && a.colmin && mn <= mx) {
            atomicMin(&a.colmin[col], mn);
            atomicMax(&a.colmax[col], mx);
        }
    }
}

// ------------------------------------------------------------ keys
// One thread per (subset, rank): grid cell of the projection, then one key
// per shifted curve. MD bounds the reduced dimension at compile time so the
// per-axis arrays stay in registers.
template <int MD>
__global__ __launch_bounds__(256) void key_kernel(KeyArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.cnt * a.S) return;
    const int s = (int)(i / a.cnt);
    const int64_t r = i - (int64_t)s * a.cnt;
    uint32_t u[MD], v[MD];
    const uint64_t sp = (uint64_t)a.span[s];
    // floor(rel (R-1) / sp) through a float64 reciprocal when the numerator
    // stays below 2^53 (rel <= sp, so the quotient is below 2^21 and off by
    // at most one, which the two integer checks correct); else the 64-bit
    // division
    const bool fdiv = a.R - 1 < (int64_t(1) << 21) && sp < (uint64_t(1) << 32);
    const double inv = 1.0 / (double)sp;
#pragma unroll
    for (int d = 0; d < MD; d++) {
        u[d] = 0;
        if (d < a.D) {
            const int64_t rel = (int64_t)a.y[r * a.ystride + s * a.D + d] - a.lo[s * a.D + d];
            uint64_t q = 0;
            if (rel > 0) {
                const uint64_t num = (uint64_t)rel * (uint64_t)(a.R - 1);
                if (fdiv && (uint64_t)rel <= sp) {
                    q = (uint64_t)((double)num * inv);
                    if (q * sp > num) q--;
                    else if ((q + 1) * sp <= num) q++;
                } else {
                    q = num / sp;
                }
            }
            if (q > (uint64_t)(a.R - 1)) q = a.R - 1;
            u[d] = (uint32_t)q;
        }
    }
    const int64_t rank = a.r0 + r;
    const uint32_t id = a.dict[rank];
    for (int j = 0; j < a.L; j++) {
        const uint32_t sh = (uint32_t)(((int64_t)j * a.R) / (a.D + 1));
#pragma unroll
        for (int d = 0; d < MD; d++) v[d] = u[d] + sh;
        if (a.curve == SFC_CURVE_HILBERT) hilbert_axes_to_transpose<MD>(v, a.D, a.b);
        uint64_t w[kMaxKeyWords];
        interleave_words<MD>(v, a.D, a.b, a.W64, w);
        const int64_t arr = (int64_t)s * a.L + j;
#pragma unroll
        for (int k = 0; k < kMaxKeyWords; k++)
            if (k < a.W64) a.keys[(arr * a.W64 + k) * a.n + rank] = w[k];
        a.ids[arr * a.n + rank] = id;
    }
}

__global__ void init_minmax_kernel(int32_t* mn, int32_t* mx, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        mn[i] = 0x7fffffff;
        mx[i] = (int32_t)0x80000000;
    }
}

// lo = column minimum; span = max(1, max_d (hi_d - lo_d)) per subset
__global__ void span_kernel(const int32_t* __restrict__ mn, const int32_t* __restrict__ mx, int S,
                            int D, int64_t* __restrict__ lo, int64_t* __restrict__ span) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int64_t sp = 1;
    for (int d = 0; d < D; d++) {
        const int64_t a = mn[s * D + d], b = mx[s * D + d];
        lo[s * D + d] = a;
        if (b - a > sp) sp = b - a;
    }
    span[s] = sp;
}

// Wt[col][e] = w_s[i][d] for col = s*D+d and e = elems_s[i]
__global__ void weights_kernel(const int8_t* __restrict__ basis, const int32_t* __restrict__ elems,
                               const int32_t* __restrict__ msz, int S, int mmax, int D, int Pk,
                               int8_t* __restrict__ Wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * mmax * D) return;
    const int s = (int)(i / ((int64_t)mmax * D));
    const int rem = (int)(i - (int64_t)s * mmax * D);
    const int r = rem / D, d = rem % D;
    if (r >= msz[s]) return;
    Wt[(int64_t)(s * D + d) * Pk + elems[s * mmax + r]] = basis[(int64_t)s * mmax * D + r * D + d];
}

// wsum[col] = 128 * sum_e Wt[col][e] (the offset the byte XOR takes away)
__global__ void weight_sums_kernel(const int8_t* __restrict__ Wt, int Pk, int cols,
                                   int32_t* __restrict__ wsum) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= cols) return;
    int sum = 0;
    for (int e = 0; e < Pk; e++) sum += Wt[(int64_t)col * Pk + e];
    wsum[col] = 128 * sum;
}

using ProjFn = void (*)(ProjArgs);
template <int NT>
ProjFn proj_fn() { return proj_kernel<NT>; }
const ProjFn kProj[] = {nullptr, proj_fn<1>(), proj_fn<2>(), proj_fn<3>(), proj_fn<4>(),
                        proj_fn<5>(), proj_fn<6>(), proj_fn<7>(), proj_fn<8>(), proj_fn<9>(),
                        proj_fn<10>(), proj_fn<11>(), proj_fn<12>(), proj_fn<13>(),
                        proj_fn<14>(), proj_fn<15>(), proj_fn<16>()};

}  // namespace

int proj_tiles(int ncols) { return (ncols + 31) / 32; }

int proj_depth(int P) { return (P + 31) / 32 * 32; }

size_t proj_weight_bytes(int ncols, int P) {
    const size_t cols = (size_t)proj_tiles(ncols) * 32;
    return cols * proj_depth(P) + cols * sizeof(int32_t);
}

sfc_status launch_weights(const int8_t* basis, const int32_t* elems, const int32_t* msz, int S,
                          int mmax, int D, int P, int ncols, int8_t* Wt, int32_t* wsum,
                          hipStream_t st) {
    const int Pk = proj_depth(P), cols = proj_tiles(ncols) * 32;
    weights_kernel<<<blocks_for((int64_t)S * mmax * D), 256, 0, st>>>(basis, elems, msz, S, mmax,
                                                                      D, Pk, Wt);
    SFC_TRY(launched("weights_kernel"));
    weight_sums_kernel<<<blocks_for(cols), 256, 0, st>>>(Wt, Pk, cols, wsum);
    return launched("weight_sums_kernel");
}

sfc_status launch_init_minmax(int32_t* mn, int32_t* mx, int n, hipStream_t st) {
    init_minmax_kernel<<<blocks_for(n), 256, 0, st>>>(mn, mx, n);
    return launched("init_minmax_kernel");
}

sfc_status launch_projection(const ProjArgs& a, hipStream_t st) {
    if (a.cnt == 0) return SFC_OK;
    const int nt = proj_tiles(a.ncols);
    if (nt < 1 || nt > 16) return fail(SFC_EUNSUPPORTED, "projection: S*D above 512 columns");
    if (a.Pk != proj_depth(a.P) || a.run < 1 || a.P % a.run != 0)
        return fail(SFC_EINVAL, "projection: inconsistent patch layout");
    const size_t lds = (size_t)kProjRows * (a.Pk + 16);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kProj[nt],
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return check_hip(e, "projection LDS attribute");
    }
    hipLaunchKernelGGL(kProj[nt], dim3(blocks_for(a.cnt, kProjRows)), dim3(256), lds, st, a);
    return launched("proj_kernel");
}

sfc_status launch_span(const int32_t* mn, const int32_t* mx, int S, int D, int64_t* lo,
                       int64_t* span, hipStream_t st) {
    span_kernel<<<blocks_for(S, 64), 64, 0, st>>>(mn, mx, S, D, lo, span);
    return launched("span_kernel");
}

sfc_status launch_keys(const KeyArgs& a, hipStream_t st) {
    if (a.cnt == 0) return SFC_OK;
    if (a.D < 1 || a.D > kMaxD) return fail(SFC_EINVAL, "keys: reduced dimension out of range");
    const unsigned nb = blocks_for(a.cnt * a.S);
    if (a.D <= 8) key_kernel<8><<<nb, 256, 0, st>>>(a);
    else if (a.D <= 16) key_kernel<16><<<nb, 256, 0, st>>>(a);
    else key_kernel<kMaxD><<<nb, 256, 0, st>>>(a);
    return launched("key_kernel");
}

}  // namespace sfc
