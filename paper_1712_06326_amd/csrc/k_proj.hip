// Index build, part 2 (Sections II.A-C): principal coordinates of every
// dictionary patch by an MFMA GEMM, their grid cells on the shifted curves
// and the curve keys.
//
// Projection: Y[n, S*D] = X[n, P] * Wcat[P, S*D], where row c of X is the
// byte-coded patch of dictionary entry c (an implicit im2col gathered from
// the quantised volume into LDS) and Wcat holds every subset's int8 basis in
// its own D columns (zero outside the subset's elements). Bytes and int8
// weights are exact in bf16 and every partial sum stays below 2^24
// (|S_s|*C <= 518), so v_mfma_f32_32x32x16_bf16 with float32 accumulation
// returns the exact integers.
#include "build.hpp"
#include "keys.hpp"
#include "proj.hpp"

namespace sfc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}

constexpr int kProjRows = 128;   // patches per workgroup (32 per wave)

__device__ inline uint32_t bf16_of_byte_pair(uint32_t w, int k) {
    // bytes k and k+1 of w -> two bf16 (upper halves of the exact floats)
    const uint32_t lo = __float_as_uint((float)((w >> (8 * k)) & 0xffu)) >> 16;
    const uint32_t hi = __float_as_uint((float)((w >> (8 * (k + 1))) & 0xffu)) >> 16;
    return lo | (hi << 16);
}

template <int NT>
__global__ __launch_bounds__(256) void proj_kernel(ProjArgs a) {
    extern __shared__ uint8_t As[];   // [kProjRows][Pp + 8]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int stride = a.Pp + 8;
    const int64_t base = (int64_t)blockIdx.x * kProjRows;
    for (int i = tid; i < kProjRows * a.Pp; i += 256) {
        const int r = i / a.Pp, e = i - r * a.Pp;
        uint8_t v = 0;
        const int64_t c = base + r;
        if (e < a.P && c < a.cnt) {
            const int64_t ctr = a.dict[a.r0 + c];
            v = a.xq[ctr * a.C + a.elem_off[e]];
        }
        As[r * stride + e] = v;
    }
    __syncthreads();
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int i = 0; i < 16; i++) acc[t][i] = 0.0f;
    const int row = wave * 32 + (lane & 31);
    const int kh = (lane >> 5) * 8;
    for (int k0 = 0; k0 < a.Pp; k0 += 16) {
        const uint8_t* ap = As + row * stride + k0 + kh;
        const uint32_t w0 = *reinterpret_cast<const uint32_t*>(ap);
        const uint32_t w1 = *reinterpret_cast<const uint32_t*>(ap + 4);
        union { uint32_t u[4]; bf16x8 v; } A;
        A.u[0] = bf16_of_byte_pair(w0, 0);
        A.u[1] = bf16_of_byte_pair(w0, 2);
        A.u[2] = bf16_of_byte_pair(w1, 0);
        A.u[3] = bf16_of_byte_pair(w1, 2);
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const uint16_t* bp = a.Wt + (int64_t)(t * 32 + (lane & 31)) * a.Pp + k0 + kh;
            union { uint4 u; bf16x8 v; } B;
            B.u = *reinterpret_cast<const uint4*>(bp);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.v, B.v, acc[t], 0, 0, 0);
        }
    }
    // epilogue: lane holds column (lane & 31) of each tile, rows
    // (i/4)*8 + (lane/32)*4 + i%4 of the wave's 32 patches.
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int col = t * 32 + (lane & 31);
        int mn = 0x7fffffff, mx = (int)0x80000000;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const int r = (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
            const int64_t c = base + wave * 32 + r;
            const int yv = (int)acc[t][i];
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
#pragma unroll
    for (int d = 0; d < MD; d++) {
        u[d] = 0;
        if (d < a.D) {
            const int64_t rel = (int64_t)a.y[r * a.ystride + s * a.D + d] - a.lo[s * a.D + d];
            uint64_t q = rel > 0 ? ((uint64_t)rel * (uint64_t)(a.R - 1)) / sp : 0;
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

// Wt[col][e] (bf16 bits) = w_s[i][d] for col = s*D+d and e = elems_s[i]
__global__ void weights_kernel(const int8_t* __restrict__ basis, const int32_t* __restrict__ elems,
                               const int32_t* __restrict__ msz, int S, int mmax, int D, int Pp,
                               uint16_t* __restrict__ Wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * mmax * D) return;
    const int s = (int)(i / ((int64_t)mmax * D));
    const int rem = (int)(i - (int64_t)s * mmax * D);
    const int r = rem / D, d = rem % D;
    if (r >= msz[s]) return;
    const float w = (float)basis[(int64_t)s * mmax * D + r * D + d];
    Wt[(int64_t)(s * D + d) * Pp + elems[s * mmax + r]] = (uint16_t)(__float_as_uint(w) >> 16);
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

sfc_status launch_weights(const int8_t* basis, const int32_t* elems, const int32_t* msz, int S,
                          int mmax, int D, int Pp, uint16_t* Wt, hipStream_t st) {
    weights_kernel<<<blocks_for((int64_t)S * mmax * D), 256, 0, st>>>(basis, elems, msz, S, mmax,
                                                                      D, Pp, Wt);
    return launched("weights_kernel");
}

sfc_status launch_init_minmax(int32_t* mn, int32_t* mx, int n, hipStream_t st) {
    init_minmax_kernel<<<blocks_for(n), 256, 0, st>>>(mn, mx, n);
    return launched("init_minmax_kernel");
}

sfc_status launch_projection(const ProjArgs& a, hipStream_t st) {
    if (a.cnt == 0) return SFC_OK;
    const int nt = proj_tiles(a.ncols);
    if (nt < 1 || nt > 16) return fail(SFC_EUNSUPPORTED, "projection: S*D above 512 columns");
    const size_t lds = (size_t)kProjRows * (a.Pp + 8);
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
