// Index query (Fig. 1 b-d): choose the subset index that best covers the
// known pixels of the target, move the query to principal space, find its
// position on each shifted curve by a wave-cooperative search, take a window
// of entries around it per curve, and rescore the union of the windows with
// the exact masked cost (a full scan in image space over the candidates).
#include "keys.hpp"
#include "loop_apply.hpp"
#include "mfma_scan.hpp"
#include "query.hpp"

namespace sfc {

namespace {

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef const __attribute__((address_space(4))) float cfloat_as4;
typedef const __attribute__((address_space(4))) uint32_t cu32_as4;
__device__ inline float ldu(const float* p) { return *(cfloat_as4*)p; }
__device__ inline uint32_t ldu(const uint32_t* p) { return *(cu32_as4*)p; }

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}

// Sums over a wave's 64 lanes, left in lane 63 (other lanes hold partial
// sums): a scan within each row of 16 lanes by DPP row shifts (lanes shifted
// in from outside the row read 0), then row_bcast:15 adds each row's total
// to the next odd row and row_bcast:31 adds lane 31 to rows 2 and 3. All in
// vector registers (no scalar register per value). Integer sums, so exact
// in any order.
__device__ inline int32_t wave_sum_i32(int32_t x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}
template <int CTRL, int ROWS, bool BOUND>
__device__ inline int64_t dpp_i64(int64_t x) {
    const uint32_t lo =
        __builtin_amdgcn_update_dpp(0u, (uint32_t)(uint64_t)x, CTRL, ROWS, 0xf, BOUND);
    const uint32_t hi =
        __builtin_amdgcn_update_dpp(0u, (uint32_t)((uint64_t)x >> 32), CTRL, ROWS, 0xf, BOUND);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline int64_t wave_sum_i64(int64_t x) {
    x += dpp_i64<0x111, 0xf, true>(x);
    x += dpp_i64<0x112, 0xf, true>(x);
    x += dpp_i64<0x114, 0xf, true>(x);
    x += dpp_i64<0x118, 0xf, true>(x);
    x += dpp_i64<0x142, 0xa, false>(x);
    x += dpp_i64<0x143, 0xc, false>(x);
    return x;
}

// Sums over each row of 16 lanes, returned to every lane of the row: a scan
// by DPP row shifts leaves the row's total in its lane 15, which a
// ds_swizzle (bit mode: lane -> (lane & 16) | 15 within each 32) copies to
// the row. Integer sums, so exact in any order.
__device__ inline int32_t row_sum_i32(int32_t x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    return __builtin_amdgcn_ds_swizzle(x, 0x01f0);   // and 0x10, or 0x0f
}
__device__ inline int64_t row_sum_i64(int64_t x) {
    x += dpp_i64<0x111, 0xf, true>(x);
    x += dpp_i64<0x112, 0xf, true>(x);
    x += dpp_i64<0x114, 0xf, true>(x);
    x += dpp_i64<0x118, 0xf, true>(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int32_t)(uint32_t)(uint64_t)x, 0x01f0);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_ds_swizzle((int32_t)(uint32_t)((uint64_t)x >> 32), 0x01f0);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane l's double, to every lane of the wave (two readlanes).
__device__ inline double bcast_f64(double x, int l) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// ------------------------------------------------------------ prologue
// G lanes per query, 256/G queries per workgroup.
//  1. The target's known pixels as a bit set (Kd <= 1024 bits), built with
//     ballots, G pixels per step.
//  2. Subset: the largest known fraction k_s/n_s, compared exactly as
//     k_a*n_b > k_b*n_a, ties to the lower subset; k_s is the popcount of the
//     known bits under the subset's pixel mask.
//  3. Over the subset's known elements, spread across the lanes: the exact
//     integer sums A = W_k^T x_k, T = W_k^T S_k and G_k = W_k^T W_k (upper
//     triangle), reduced across the group (integer sums: any order).
//  4. The least-squares imputation of the unknown elements, from
//       G z = r,  G = G_k + I,  r = n_sub A - T           (integers)
//     by Gaussian elimination without pivoting in float64 (column by
//     column, then back substitution), and
//       y_d = A_d + (B_d + sum_e H_de z_e) / n_sub,
//       B = W^T S - T = W_u^T S_u,  H = W^T W - G_k = W_u^T W_u.
//     Every lane of the group computes this in the same order (no lane
//     exchanges in float64).
//  5. The grid cell, then one key per shifted curve (lane j: curve j).
constexpr int kPrologueLanes = 16;
constexpr int64_t kPrologueWideQ = 256;   // up to this many queries: a workgroup per query
constexpr int kMaxKnownWords = 16;   // K^nd <= 1024
constexpr int kMaxSubsets = 26;      // 3^3 - 1

template <int D, int G>
__global__ __launch_bounds__(256) void prologue_kernel(QueryIndexView v, const float* __restrict__ t,
                                                       const uint8_t* __restrict__ m, int64_t Q,
                                                       int32_t* __restrict__ qsub,
                                                       double* __restrict__ qcoords,
                                                       uint64_t* __restrict__ qkeys,
                                                       uint32_t* __restrict__ rowmask,
                                                       int64_t qpad) {
    static_assert(64 % G == 0 && G >= 4, "a group of lanes lies inside one wave");
    constexpr int NG = 256 / G;
    constexpr int NT = D * (D + 1) / 2;
    __shared__ uint64_t known_bits[NG][kMaxKnownWords];
    __shared__ int32_t known_cnt[NG][kMaxSubsets];
    const int lane = threadIdx.x & 63;
    const int grp = threadIdx.x / G;
    const int gl = threadIdx.x % G;
    const int64_t q = (int64_t)blockIdx.x * NG + grp;
    const bool live = q < Q;
    // a group past the end shadows the last query (every lane takes part in
    // the ballots) and stores nothing
    const int64_t qq = live ? q : Q - 1;
    const uint8_t* mq = m + qq * v.Kd;
    const float* tq = t + qq * (int64_t)v.Kd * v.C;
    const int KW = (v.Kd + 63) >> 6;
    const int gshift = (lane / G) * G;
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);

    // 1. known bits
    for (int w = 0; w < KW; w++) {
        uint64_t word = 0;
        for (int sub = 0; sub < 64; sub += G) {
            const int p = w * 64 + sub + gl;
            const bool k = p < v.Kd && mq[p] != 0;
            word |= ((__ballot(k) >> gshift) & gmask) << sub;
        }
        if (gl == 0) known_bits[grp][w] = word;
    }
    __syncthreads();

    // the rescoring's row masks: bit dx of row r = pixel r*K + dx known
    if (rowmask && live) {
        for (int r = gl; r < v.rows; r += G) {
            const int p0 = r * v.K;
            const int w0 = p0 >> 6, b0 = p0 & 63;
            uint64_t bits = known_bits[grp][w0] >> b0;
            if (b0 + v.K > 64) bits |= known_bits[grp][w0 + 1] << (64 - b0);
            rowmask[(int64_t)r * qpad + q] = (uint32_t)(bits & ((1ull << v.K) - 1ull));
        }
    }

    // 2. subset choice
    for (int s = gl; s < v.S; s += G) {
        int k = 0;
        for (int w = 0; w < KW; w++) k += __popcll(known_bits[grp][w] & v.smask[s * KW + w]);
        known_cnt[grp][s] = k;
    }
    __syncthreads();
    int sb = 0;
    int64_t kb = -1, nbest = 1;
    for (int s = 0; s < v.S; s++) {
        const int64_t k = known_cnt[grp][s], ns = v.npix[s];
        if (kb < 0 || k * nbest > kb * ns) {
            sb = s;
            kb = k;
            nbest = ns;
        }
    }

    // 3. exact sums over the known elements
    int32_t A[D], Gk[NT];
    int64_t T[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        A[d] = 0;
        T[d] = 0;
    }
#pragma unroll
    for (int i = 0; i < NT; i++) Gk[i] = 0;
    const float vmin = v.qparams[0], sc = v.qparams[1];
    const int8_t* wb = v.basis + (int64_t)sb * v.mmax * D;
    const int np = v.npix[sb];
    for (int i = gl; i < np; i += G) {
        const int rho = v.pix[sb * v.Kd + i];
        if (!((known_bits[grp][rho >> 6] >> (rho & 63)) & 1ull)) continue;
        for (int ch = 0; ch < v.C; ch++) {
            const int e = rho * v.C + ch;
            float rr = __builtin_rintf((tq[e] - vmin) * sc);
            if (!(rr >= 0.0f)) rr = 0.0f;
            if (rr > 255.0f) rr = 255.0f;
            const int32_t x = (int32_t)rr;
            const int64_t se = (int64_t)v.sum[e];
            const int8_t* wr = wb + (int64_t)(i * v.C + ch) * D;
            int32_t w[D];
#pragma unroll
            for (int d = 0; d < D; d++) w[d] = wr[d];
            int k = 0;
#pragma unroll
            for (int d = 0; d < D; d++) {
                A[d] += w[d] * x;
                T[d] += (int64_t)w[d] * se;
#pragma unroll
                for (int f = d; f < D; f++) Gk[k++] += w[d] * w[f];
            }
        }
    }
    if (G == 16) {   // a query's group is one DPP row
#pragma unroll
        for (int d = 0; d < D; d++) {
            A[d] = row_sum_i32(A[d]);
            T[d] = row_sum_i64(T[d]);
        }
#pragma unroll
        for (int i = 0; i < NT; i++) Gk[i] = row_sum_i32(Gk[i]);
    } else {
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
#pragma unroll
            for (int d = 0; d < D; d++) {
                A[d] += __shfl_xor(A[d], off, 64);
                T[d] += (int64_t)__shfl_xor((long long)T[d], off, 64);
            }
#pragma unroll
            for (int i = 0; i < NT; i++) Gk[i] += __shfl_xor(Gk[i], off, 64);
        }
    }

    // 4. imputation in float64, the oracle's order, one row per lane of the
    // group (D <= 16 = G): lane r holds row r of G_k + I and r_r; each
    // pivot step shares the pivot row within the group and the rows below
    // it apply the serial elimination's operations to themselves, in its
    // order; back substitution stays serial, lane d forms y_d (lanes from D
    // on mirror row D - 1 and are never read)
    static_assert(G == 16 && D <= G, "one row per lane of a 16-lane group");
    const int64_t* wtw = v.wtw + (int64_t)sb * D * D;
    const int64_t* ws = v.ws + (int64_t)sb * D;
    const int row = gl < D ? gl : D - 1;
    int32_t Ar = 0, grow[D];
    int64_t Tr = 0;
#pragma unroll
    for (int f = 0; f < D; f++) grow[f] = 0;
#pragma unroll
    for (int r = 0; r < D; r++) {
        if (row != r) continue;
        Ar = A[r];
        Tr = T[r];
#pragma unroll
        for (int f = 0; f < D; f++) {
            const int lo = r < f ? r : f, hi = r < f ? f : r;
            grow[f] = Gk[lo * D - lo * (lo - 1) / 2 + (hi - lo)];
        }
    }
    double ai[D], ri;
#pragma unroll
    for (int f = 0; f < D; f++) {
        // |entries of W^T W and G_k| <= 128^2 * (1024 * 16) = 2^28:
        // exact through a 32-bit conversion
        ai[f] = (double)(grow[f] + (row == f ? 1 : 0));
    }
    ri = (double)(v.nsub * (int64_t)Ar - Tr);
#pragma unroll
    for (int k = 0; k < D; k++) {
        const double akk = __shfl(ai[k], k, G), rk = __shfl(ri, k, G);
        double akj[D];
#pragma unroll
        for (int jj = k + 1; jj < D; jj++) akj[jj] = __shfl(ai[jj], k, G);
        if (row > k) {
            const double fct = ai[k] / akk;
#pragma unroll
            for (int jj = k + 1; jj < D; jj++) ai[jj] = ai[jj] - fct * akj[jj];
            ri = ri - fct * rk;
        }
    }
    double z[D];
#pragma unroll
    for (int r = D - 1; r >= 0; r--) {
        double zr = 0.0;
        if (gl == r) {
            double sacc = ri;
#pragma unroll
            for (int jj = r + 1; jj < D; jj++) sacc = sacc - ai[jj] * z[jj];
            zr = sacc / ai[r];
        }
        z[r] = __shfl(zr, r, G);
    }
    double yd;
    {
        double f = (double)(ws[row] - Tr);
#pragma unroll
        for (int e = 0; e < D; e++)
            f = f + (double)(int32_t)(wtw[row * D + e] - (int64_t)grow[e]) * z[e];
        yd = (double)Ar + f / (double)v.nsub;
    }
    double y[D];
#pragma unroll
    for (int d = 0; d < D; d++) y[d] = __shfl(yd, d, G);
    if (!live) return;
    if (gl == 0) {
        qsub[q] = sb;
#pragma unroll
        for (int d = 0; d < D; d++) qcoords[q * D + d] = y[d];
    }

    // 5. grid cell and one key per shifted curve
    const double span = (double)v.span[sb];
    const double rm1 = (double)(v.R - 1);
    uint32_t u[D], cell[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        double uu = floor(((y[d] - (double)v.lo[sb * D + d]) * rm1) / span);
        if (!(uu >= 0.0)) uu = 0.0;
        if (uu > rm1) uu = rm1;
        u[d] = (uint32_t)(int64_t)uu;
    }
    for (int j = gl; j < v.L; j += G) {
        const uint32_t sh = (uint32_t)(((int64_t)j * v.R) / (D + 1));
#pragma unroll
        for (int d = 0; d < D; d++) cell[d] = u[d] + sh;
        if (v.curve == SFC_CURVE_HILBERT) hilbert_axes_to_transpose<D>(cell, D, v.b);
        uint64_t w[kMaxKeyWords];
        interleave_words<D>(cell, D, v.b, v.W64, w);
        for (int k = 0; k < v.W64; k++) qkeys[(q * v.L + j) * v.W64 + k] = w[k];
    }
}

// One query per workgroup of 256 threads, for small batches (the fill
// loop's lone target): the steps and arithmetic of prologue_kernel, laid
// out so that every phase issues all of its global loads before it uses
// one. A query then waits for a few memory round trips (mask and subset
// masks; pixel list; element values) instead of one per known word, per
// subset and per group of G pixels. The subset is chosen by a tournament
// over the lanes under the same total order (larger k_s/n_s first, then
// the lower index). With qbest non-null the query's packed best and its
// ticket counter are cleared for the split rescoring.
template <int D>
__global__ __launch_bounds__(256) void prologue_one_kernel(
    QueryIndexView v, const float* __restrict__ t, const uint8_t* __restrict__ m, int64_t Q,
    int32_t* __restrict__ qsub, double* __restrict__ qcoords, uint64_t* __restrict__ qkeys,
    uint32_t* __restrict__ rowmask, int64_t qpad, uint64_t* __restrict__ qbest,
    int32_t* __restrict__ qticket) {
    constexpr int NT = D * (D + 1) / 2;
    constexpr int NV = 3 * D + NT;   // A, T (two words each), G_k
    __shared__ uint64_t kbits[kMaxKnownWords];
    __shared__ int32_t kcnt[32], knp[32];
    __shared__ int32_t red[4][NV];
    __shared__ int64_t swtw[D * D], sws[D], slo[D];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t q = blockIdx.x;
    if (q >= Q) return;   // uniform: the grid is Q workgroups
    const int KW = (v.Kd + 63) >> 6;
    const int SW = v.S * KW;
    const uint8_t* mq = m + q * v.Kd;
    const float* tq = t + q * (int64_t)v.Kd * v.C;

    // 1. known bits (Kd <= 1024: four bytes per thread), the subsets' pixel
    // masks (S * KW <= 416 words: two per thread) and sizes, all at once
    uint8_t mb[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int p = tid + 256 * k;
        mb[k] = mq[p < v.Kd ? p : 0];
    }
    uint64_t smw[2];
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const int i = tid + 256 * k;
        smw[k] = v.smask[i < SW ? i : 0];
    }
    const int32_t npx = v.npix[tid < v.S ? tid : 0];
    if (tid < 32) kcnt[tid] = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int p = tid + 256 * k;   // word 4k + wave, bit lane
        const uint64_t word = __ballot(p < v.Kd && mb[k] != 0);
        if (lane == 0 && 4 * k + wave < KW) kbits[4 * k + wave] = word;
    }
    if (tid < v.S) knp[tid] = npx;
    __syncthreads();

    // the rescoring's row masks: bit dx of row r = pixel r*K + dx known
    if (rowmask) {
        for (int r = tid; r < v.rows; r += 256) {
            const int p0 = r * v.K;
            const int w0 = p0 >> 6, b0 = p0 & 63;
            uint64_t bits = kbits[w0] >> b0;
            if (b0 + v.K > 64) bits |= kbits[w0 + 1] << (64 - b0);
            rowmask[(int64_t)r * qpad + q] = (uint32_t)(bits & ((1ull << v.K) - 1ull));
        }
    }
    // 2. known pixels of each subset (exact integer counts)
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const int i = tid + 256 * k;
        if (i < SW) {
            const int c = __popcll(kbits[i % KW] & smw[k]);
            if (c) atomicAdd(&kcnt[i / KW], c);
        }
    }
    __syncthreads();
    int32_t kk = -1, nn = 1, ss = lane;   // lanes >= S lose every comparison
    if (lane < v.S) {
        kk = kcnt[lane];
        nn = knp[lane];
    }
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const int32_t ko = __shfl_xor(kk, off, 64), no = __shfl_xor(nn, off, 64),
                      so = __shfl_xor(ss, off, 64);
        const int64_t l = (int64_t)ko * nn, r = (int64_t)kk * no;
        if (l > r || (l == r && so < ss)) {
            kk = ko;
            nn = no;
            ss = so;
        }
    }
    const int sb = __builtin_amdgcn_readfirstlane(ss);

    // the subset's constants, loaded now and used after the sums
    const int64_t wv = v.wtw[(int64_t)sb * D * D + (tid < D * D ? tid : 0)];
    const int64_t wsv = v.ws[(int64_t)sb * D + (tid < D ? tid : 0)];
    const int64_t lov = v.lo[(int64_t)sb * D + (tid < D ? tid : 0)];
    const int64_t spv = v.span[sb];

    // 3. exact sums over the subset's known elements; element j is pixel
    // j / C of the subset, channel j % C, and row j of its basis
    int32_t A[D], Gk[NT];
    int64_t T[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        A[d] = 0;
        T[d] = 0;
    }
#pragma unroll
    for (int i = 0; i < NT; i++) Gk[i] = 0;
    const float vmin = v.qparams[0], sc = v.qparams[1];
    const int8_t* wb = v.basis + (int64_t)sb * v.mmax * D;
    const int32_t* pixs = v.pix + (int64_t)sb * v.Kd;
    const int C = v.C;
    const int ne = knp[sb] * C;
    for (int base = 0; base < ne; base += 512) {
        int rho[2];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int j = base + tid + 256 * u;
            rho[u] = pixs[(j < ne ? j : 0) / C];
        }
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int j = base + tid + 256 * u;
            const bool ok = j < ne && ((kbits[rho[u] >> 6] >> (rho[u] & 63)) & 1ull);
            const int jc = ok ? j : 0;
            const int e = (ok ? rho[u] : 0) * C + jc % C;
            float rr = __builtin_rintf((tq[e] - vmin) * sc);
            if (!(rr >= 0.0f)) rr = 0.0f;
            if (rr > 255.0f) rr = 255.0f;
            const int32_t x = (int32_t)rr;
            const int64_t se = (int64_t)v.sum[e];
            const int8_t* wr = wb + (int64_t)jc * D;
            int32_t w[D];
#pragma unroll
            for (int d = 0; d < D; d++) w[d] = ok ? (int32_t)wr[d] : 0;
            int k = 0;
#pragma unroll
            for (int d = 0; d < D; d++) {
                A[d] += w[d] * x;
                T[d] += (int64_t)w[d] * se;
#pragma unroll
                for (int f = d; f < D; f++) Gk[k++] += w[d] * w[f];
            }
        }
    }
#pragma unroll
    for (int d = 0; d < D; d++) {
        A[d] = wave_sum_i32(A[d]);
        T[d] = wave_sum_i64(T[d]);
    }
#pragma unroll
    for (int i = 0; i < NT; i++) Gk[i] = wave_sum_i32(Gk[i]);
    if (lane == 63) {   // the wave's totals
#pragma unroll
        for (int d = 0; d < D; d++) {
            red[wave][d] = A[d];
            red[wave][D + 2 * d] = (int32_t)(uint32_t)(uint64_t)T[d];
            red[wave][D + 2 * d + 1] = (int32_t)(uint32_t)((uint64_t)T[d] >> 32);
        }
#pragma unroll
        for (int i = 0; i < NT; i++) red[wave][3 * D + i] = Gk[i];
    }
    if (tid < D * D) swtw[tid] = wv;
    if (tid < D) {
        sws[tid] = wsv;
        slo[tid] = lov;
    }
    __syncthreads();
    // waves without a curve to key have nothing left to do
    if (wave > 0 && wave * 64 >= v.L) return;
#pragma unroll
    for (int d = 0; d < D; d++) {
        A[d] = red[0][d] + red[1][d] + red[2][d] + red[3][d];
        uint64_t tt = 0;
#pragma unroll
        for (int k = 0; k < 4; k++)
            tt += (uint64_t)(uint32_t)red[k][D + 2 * d] |
                  ((uint64_t)(uint32_t)red[k][D + 2 * d + 1] << 32);
        T[d] = (int64_t)tt;
    }
#pragma unroll
    for (int i = 0; i < NT; i++)
        Gk[i] = red[0][3 * D + i] + red[1][3 * D + i] + red[2][3 * D + i] + red[3][3 * D + i];

    // 4. imputation in float64, the oracle's order, one row per lane: lane i
    // < D holds row i of G_k + I and r_i; each pivot step broadcasts the
    // pivot row (readlane) and the rows below it update themselves with the
    // operations the serial elimination applies to them, in its order
    // (lanes from D on mirror row D - 1 and are never read)
    __shared__ int64_t stot[2 * D + NT];   // A, T, G_k
    if (tid == 0) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            stot[d] = A[d];
            stot[D + d] = T[d];
        }
#pragma unroll
        for (int k = 0; k < NT; k++) stot[2 * D + k] = Gk[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int row = lane < D ? lane : D - 1;
    double ai[D], ri;
#pragma unroll
    for (int f = 0; f < D; f++) {
        const int lo = row < f ? row : f, hi = row < f ? f : row;
        const int k = lo * D - lo * (lo - 1) / 2 + (hi - lo);
        ai[f] = (double)((int32_t)stot[2 * D + k] + (row == f ? 1 : 0));
    }
    ri = (double)(v.nsub * stot[row] - stot[D + row]);
#pragma unroll
    for (int k = 0; k < D; k++) {
        const double akk = bcast_f64(ai[k], k), rk = bcast_f64(ri, k);
        double akj[D];
#pragma unroll
        for (int jj = k + 1; jj < D; jj++) akj[jj] = bcast_f64(ai[jj], k);
        if (row > k) {
            const double fct = ai[k] / akk;
#pragma unroll
            for (int jj = k + 1; jj < D; jj++) ai[jj] = ai[jj] - fct * akj[jj];
            ri = ri - fct * rk;
        }
    }
    // back substitution, rows from the last: lane i finishes z_i, all take it
    double z[D];
#pragma unroll
    for (int r = D - 1; r >= 0; r--) {
        double zr = 0.0;
        if (lane == r) {
            double sacc = ri;
#pragma unroll
            for (int jj = r + 1; jj < D; jj++) sacc = sacc - ai[jj] * z[jj];
            zr = sacc / ai[r];
        }
        z[r] = bcast_f64(zr, r);
    }
    // y_d on lane d, then to every lane
    double yd;
    {
        const int d = row;
        double f = (double)(sws[d] - stot[D + d]);
#pragma unroll
        for (int e = 0; e < D; e++) {
            const int lo = d < e ? d : e, hi = d < e ? e : d;
            const int k = lo * D - lo * (lo - 1) / 2 + (hi - lo);
            f = f + (double)(int32_t)(swtw[d * D + e] - stot[2 * D + k]) * z[e];
        }
        yd = (double)stot[d] + f / (double)v.nsub;
    }
    double y[D];
#pragma unroll
    for (int d = 0; d < D; d++) y[d] = bcast_f64(yd, d);
    if (tid == 0) {
        qsub[q] = sb;
#pragma unroll
        for (int d = 0; d < D; d++) qcoords[q * D + d] = y[d];
        if (qbest) {
            qbest[q] = ~0ull;
            qticket[q] = 0;
        }
    }

    // 5. grid cell and one key per shifted curve
    const double span = (double)spv;
    const double rm1 = (double)(v.R - 1);
    uint32_t u[D], cell[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        double uu = floor(((y[d] - (double)slo[d]) * rm1) / span);
        if (!(uu >= 0.0)) uu = 0.0;
        if (uu > rm1) uu = rm1;
        u[d] = (uint32_t)(int64_t)uu;
    }
    for (int j = tid; j < v.L; j += 256) {
        const uint32_t sh = (uint32_t)(((int64_t)j * v.R) / (D + 1));
#pragma unroll
        for (int d = 0; d < D; d++) cell[d] = u[d] + sh;
        if (v.curve == SFC_CURVE_HILBERT) hilbert_axes_to_transpose<D>(cell, D, v.b);
        uint64_t w[kMaxKeyWords];
        interleave_words<D>(cell, D, v.b, v.W64, w);
        for (int k = 0; k < v.W64; k++) qkeys[(q * v.L + j) * v.W64 + k] = w[k];
    }
}

// ------------------------------------------------------------ search
// Words are read only while the higher ones tie: the first word almost
// always decides, and loading every word up front measured twice as slow.
__device__ inline bool key_less(const uint64_t* K, int64_t n, int64_t pos, const uint64_t* qk,
                                int W64) {
    for (int w = 0; w < W64; w++) {
        const uint64_t a = K[(int64_t)w * n + pos];
        if (a != qk[w]) return a < qk[w];
    }
    return false;
}

// First position whose key is >= the query key, for each (query, curve),
// by G lanes: rounds of G probes split the interval into G + 1 parts (a
// ballot gives the number of probes below the key), then a final round over
// <= G entries; the window starts half a window before it, clamped. G = 64
// is one wave per search (fewest rounds, for small batches); G = 16 puts
// four searches in a wave, so that a large batch's searches are all resident
// at once.
template <int G>
__global__ __launch_bounds__(256) void search_kernel(QueryIndexView v, const int32_t* __restrict__ qsub,
                                                     const uint64_t* __restrict__ qkeys, int64_t Q,
                                                     int64_t* __restrict__ wstart) {
    const int lane = threadIdx.x & 63;
    const int sl = lane % G, grp = lane / G;
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;   // search index
    const int64_t wave0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 / G);
    if (wave0 >= Q * v.L) return;   // uniform over the wave
    const bool live = wid < Q * v.L;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1) << (grp * G));
    int64_t q = 0;
    int j = 0;
    if (live) {
        q = wid / v.L;
        j = (int)(wid - q * v.L);
    }
    const int s = live ? qsub[q] : 0;
    const uint64_t* K = v.keys + ((int64_t)s * v.L + j) * v.W64 * v.n;
    uint64_t qk[kMaxKeyWords];
    for (int w = 0; w < v.W64; w++) qk[w] = live ? qkeys[(q * v.L + j) * v.W64 + w] : 0;
    int64_t a = 0, z = live ? v.n : 0;
    // every group takes part in every ballot; a finished group probes nothing
    bool more = __ballot(z - a > G) != 0;
    while (more) {
        const int64_t len = z - a;
        const bool act = len > G;
        const int64_t pos = a + ((int64_t)(sl + 1) * len) / (G + 1);
        const bool less = act && key_less(K, v.n, pos, qk, v.W64);
        const int cnt = __popcll(__ballot(less) & gmask);
        if (act) {
            const int64_t na = cnt > 0 ? a + ((int64_t)cnt * len) / (G + 1) + 1 : a;
            const int64_t nz = cnt < G ? a + ((int64_t)(cnt + 1) * len) / (G + 1) : z;
            a = na;
            z = nz;
        }
        more = __ballot(z - a > G) != 0;
    }
    const int64_t len = z - a;
    const bool less = live && sl < len && key_less(K, v.n, a + sl, qk, v.W64);
    const int64_t p = a + __popcll(__ballot(less) & gmask);
    int64_t lo = p - v.window / 2;
    int64_t lmax = v.n - v.window;
    if (lmax < 0) lmax = 0;
    if (lo > lmax) lo = lmax;
    if (lo < 0) lo = 0;
    if (live && sl == 0) wstart[wid] = lo;
}

// ------------------------------------------------------------ rescore
constexpr int kCap = 2048;   // maximum L*W
constexpr int64_t kRescoreSharedQ = 512;   // up to this many queries: a workgroup per query
constexpr int64_t kRescoreSplitQ = 32;     // up to this many: several workgroups per query
constexpr int64_t kSplitShareBytes = 16384;   // patch bytes per workgroup of the split
static_assert(kRescoreSplitQ <= kPrologueWideQ, "the one-query prologue clears the split's words");

// Rows of a patch whose loads a lone query's cost requests together: about
// 84 floats of them.
constexpr int cost_row_group(int ND, int K, int C) {
    const int rows = ND == 2 ? K : K * K, g = 84 / (K * C);
    return g < 1 ? 1 : (g > rows ? rows : g);
}

template <int ND, int K, int C, int NORM, int RB = 1>
__device__ inline float cand_cost(const QueryIndexView& v, const float* __restrict__ vol,
                                  const float* __restrict__ tq, const uint32_t* __restrict__ rm,
                                  int64_t qpad, uint32_t c) {
    constexpr int H = (K - 1) / 2;
    constexpr int ROWS = (ND == 2) ? K : K * K;
    constexpr int RW = K * C;
    // RB rows are requested together (all their loads before the first
    // sum): a lone query then waits for ROWS / RB memory round trips
    // instead of ROWS, at the price of RB rows of registers
    float acc = 0.0f;
    for (int r0 = 0; r0 < ROWS; r0 += RB) {
        uint32_t mrs[RB];
        float vv[RB][RW];
#pragma unroll
        for (int k = 0; k < RB; k++) mrs[k] = (r0 + k < ROWS) ? ldu(rm + (int64_t)(r0 + k) * qpad) : 0u;
        // the group's rows that hold a known pixel, K*C floats each by
        // 16-byte loads at 4-byte alignment (global loads of this width
        // need only dword alignment)
#pragma unroll
        for (int k = 0; k < RB; k++) {
            const int r = r0 + k;
            if (mrs[k] == 0) continue;
            int64_t roff;
            if (ND == 2) roff = (int64_t)(r - H) * v.stride[0] - H;
            else roff = (int64_t)(r / K - H) * v.stride[0] + (int64_t)(r % K - H) * v.stride[1] - H;
            const float* vp = vol + ((int64_t)c + roff) * C;
            const f4u* vp4 = reinterpret_cast<const f4u*>(vp);
#pragma unroll
            for (int i = 0; i < RW / 4; i++) {
                const f4u x = vp4[i];
                vv[k][4 * i] = x.x;
                vv[k][4 * i + 1] = x.y;
                vv[k][4 * i + 2] = x.z;
                vv[k][4 * i + 3] = x.w;
            }
#pragma unroll
            for (int i = (RW / 4) * 4; i < RW; i++) vv[k][i] = vp[i];
        }
        // then the costs, rows ascending, pixels and channels ascending
#pragma unroll
        for (int k = 0; k < RB; k++) {
            const uint32_t mr = mrs[k];
            if (mr == 0) continue;
            const float* tp = tq + (int64_t)(r0 + k) * RW;
#pragma unroll
            for (int dx = 0; dx < K; dx++) {
                if (mr & (1u << dx)) {
#pragma unroll
                    for (int ch = 0; ch < C; ch++) {
                        const float d = ldu(tp + dx * C + ch) - vv[k][dx * C + ch];
                        // d*d fused (L2) or |d| added (L1, Section III.K)
                        if (NORM == 0) acc = __builtin_fmaf(d, d, acc);
                        else acc = acc + __builtin_fabsf(d);
                    }
                }
            }
        }
    }
    return acc;
}

// One wave per query: gather the window ids, sort them in LDS (bitonic),
// keep the unique ones, then each lane rescores every 64th candidate.
template <int ND, int K, int C, int NORM, int RB = 1>
__global__ __launch_bounds__(256) void rescore_kernel(QueryIndexView v, const float* __restrict__ vol,
                                                      const float* __restrict__ t,
                                                      const uint32_t* __restrict__ rowmask,
                                                      int64_t qpad, const int32_t* __restrict__ qsub,
                                                      const int64_t* __restrict__ wstart, int64_t Q,
                                                      int cap, int64_t* __restrict__ best_id,
                                                      float* __restrict__ best_cost,
                                                      int64_t* __restrict__ cand,
                                                      int32_t* __restrict__ ncand, int wpq) {
    // per wave: cap ids to sort (A), then the unique ones (Bu); cap is the
    // power of two >= L*W, so the launch sizes the LDS to 2 * 4 * cap words
    extern __shared__ uint32_t rescore_lds[];
    __shared__ uint64_t wbest[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // XCD-aware: workgroup b runs on XCD b % 8; each XCD takes one
    // contiguous eighth of the queries, whose neighbouring targets share
    // candidates, so the patches they gather stay in that XCD's L2.
    // wpq = 1: four queries per workgroup, one wave each; wpq = 4 (few
    // queries): the four waves share one query (each builds the same
    // candidate set) and split its candidates.
    const int64_t nblk = gridDim.x, per_xcd = (nblk + 7) / 8;
    const int64_t qb = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int64_t q = wpq == 4 ? qb : qb * 4 + w;
    const bool live = q < Q;
    const int LW = v.L * v.window;
    const int s = live ? qsub[q] : 0;
    if (!cand) {
        // Best answer only: the windows' ids go into a hash set in LDS (2 cap
        // slots per query, linear probing by compare-and-swap) and the thread
        // that inserts an id rescores it, so every distinct candidate is
        // costed once, after a single barrier. The (cost, id) minimum does
        // not depend on who costs what.
        const int T = 2 * cap;   // a power of two, at least 2 L W
        uint32_t* tab = rescore_lds + (size_t)(wpq == 4 ? 0 : w) * T;
        const int gsz = 64 * wpq, gid = wpq == 4 ? (int)threadIdx.x : lane;
        for (int i = gid; i < T; i += gsz) tab[i] = 0xffffffffu;
        __syncthreads();
        uint64_t best = ~0ull;
        if (live) {
            const float* tq = t + q * (int64_t)v.Kd * C;
            const uint32_t* rm = rowmask + q;
            const int shift = 32 - __builtin_ctz((unsigned)T);
            for (int i = gid; i < LW; i += gsz) {
                const int j = i / v.window, k = i - j * v.window;
                const int64_t pos = wstart[q * v.L + j] + k;
                if (pos >= v.n) continue;
                const uint32_t id = v.ids[((int64_t)s * v.L + j) * v.n + pos];
                uint32_t h = (id * 0x9E3779B1u) >> shift;
                bool mine = false;
                while (true) {   // ends: at most LW of the T >= 2 LW slots are taken
                    const uint32_t old = atomicCAS(&tab[h], 0xffffffffu, id);
                    if (old == 0xffffffffu) {
                        mine = true;
                        break;
                    }
                    if (old == id) break;
                    h = (h + 1) & (uint32_t)(T - 1);
                }
                if (mine) {
                    const float cost = cand_cost<ND, K, C, NORM, RB>(v, vol, tq, rm, qpad, id);
                    const uint64_t pk = ((uint64_t)__float_as_uint(cost) << 32) | id;
                    if (pk < best) best = pk;
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = (uint64_t)__shfl_xor((long long)best, off, 64);
            if (o < best) best = o;
        }
        if (wpq == 4) {
            if (lane == 0) wbest[w] = best;
            __syncthreads();
            if (w != 0) return;
            for (int k = 1; k < 4; k++) best = wbest[k] < best ? wbest[k] : best;
        }
        if (!live || !best_id) return;
        if (lane == 0) {
            best_id[q] = best == ~0ull ? -1 : (int64_t)(best & 0xffffffffull);
            best_cost[q] = best == ~0ull ? __builtin_inff() : __uint_as_float((uint32_t)(best >> 32));
        }
        return;
    }
    uint32_t* A = rescore_lds + (size_t)w * cap;
    uint32_t* Bu = rescore_lds + (size_t)(4 + w) * cap;
    for (int i = lane; i < cap; i += 64) {
        uint32_t id = 0xffffffffu;
        if (live && i < LW) {
            const int j = i / v.window, k = i - j * v.window;
            const int64_t pos = wstart[q * v.L + j] + k;
            if (pos < v.n) id = v.ids[((int64_t)s * v.L + j) * v.n + pos];
        }
        A[i] = id;
    }
    __syncthreads();
    for (int size = 2; size <= cap; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = lane; i < cap / 2; i += 64) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint32_t x = A[lo], y = A[hi];
                if ((x > y) == up) {
                    A[lo] = y;
                    A[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    int nu = 0;
    for (int base = 0; base < cap; base += 64) {
        const int i = base + lane;
        const uint32_t x = A[i];
        const bool keep = x != 0xffffffffu && (i == 0 || A[i - 1] != x);
        const uint64_t bal = __ballot(keep);
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if (keep) Bu[nu + __popcll(bal & lt)] = x;
        nu += __popcll(bal);
    }
    __syncthreads();
    if (!live) return;   // uniform over the workgroup when wpq = 4
    const bool lead = wpq == 1 || w == 0;
    if (cand && lead) {
        for (int i = lane; i < LW; i += 64) cand[q * LW + i] = i < nu ? (int64_t)Bu[i] : -1;
        if (lane == 0) ncand[q] = nu;
    }
    if (!best_id) return;
    const float* tq = t + q * (int64_t)v.Kd * C;
    const uint32_t* rm = rowmask + q;
    uint64_t best = ~0ull;
    for (int i = (wpq == 4 ? w * 64 : 0) + lane; i < nu; i += 64 * wpq) {
        const uint32_t c = Bu[i];
        const float cost = cand_cost<ND, K, C, NORM, RB>(v, vol, tq, rm, qpad, c);
        const uint64_t pk = ((uint64_t)__float_as_uint(cost) << 32) | c;
        if (pk < best) best = pk;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((long long)best, off, 64);
        if (o < best) best = o;
    }
    if (wpq == 4) {
        if (lane == 0) wbest[w] = best;
        __syncthreads();
        if (w != 0) return;
        for (int k = 1; k < 4; k++) best = wbest[k] < best ? wbest[k] : best;
    }
    if (lane == 0) {
        best_id[q] = best == ~0ull ? -1 : (int64_t)(best & 0xffffffffull);
        best_cost[q] = best == ~0ull ? __builtin_inff() : __uint_as_float((uint32_t)(best >> 32));
    }
}

// Rows of a candidate requested together by the split rescoring, where a
// thread costs a single candidate and a query has few workgroups, so
// occupancy does not matter: up to 248 floats (a whole 9x9x3 or 5x5x5x2
// patch; the 7x7x7 one in two groups), as many as the registers hold
// without spilling, balanced over the groups.
constexpr int split_row_group(int ND, int K, int C) {
    const int rows = ND == 2 ? K : K * K;
    int g = 248 / (K * C);
    g = g < 1 ? 1 : (g > rows ? rows : g);
    const int groups = (rows + g - 1) / g;
    return (rows + groups - 1) / groups;
}

// The masked cost of candidate c against a target (st: K^nd * C floats) and
// row masks (srm) staged in LDS, for the split rescoring: every row of the
// patch is requested at once (RB rows at a time; all lie inside the volume)
// and the terms are added in cand_cost's order (rows ascending, pixels and
// channels ascending), an unknown pixel's difference masked to +0, which
// leaves the sum unchanged.
template <int ND, int K, int C, int NORM, int RB>
__device__ inline float staged_cost(const QueryIndexView& v, const float* __restrict__ vol,
                                    const float* st, const uint32_t* srm, uint32_t c) {
    constexpr int H = (K - 1) / 2;
    constexpr int ROWS = (ND == 2) ? K : K * K;
    constexpr int RW = K * C;
    float acc = 0.0f;
    for (int r0 = 0; r0 < ROWS; r0 += RB) {
        float vv[RB][RW];
#pragma unroll
        for (int k = 0; k < RB; k++) {
            const int r = r0 + k;
            if (r >= ROWS) continue;
            int64_t roff;
            if (ND == 2) roff = (int64_t)(r - H) * v.stride[0] - H;
            else roff = (int64_t)(r / K - H) * v.stride[0] + (int64_t)(r % K - H) * v.stride[1] - H;
            const float* vp = vol + ((int64_t)c + roff) * C;
            const f4u* vp4 = reinterpret_cast<const f4u*>(vp);
#pragma unroll
            for (int i = 0; i < RW / 4; i++) {
                const f4u x = vp4[i];
                vv[k][4 * i] = x.x;
                vv[k][4 * i + 1] = x.y;
                vv[k][4 * i + 2] = x.z;
                vv[k][4 * i + 3] = x.w;
            }
#pragma unroll
            for (int i = (RW / 4) * 4; i < RW; i++) vv[k][i] = vp[i];
        }
#pragma unroll
        for (int k = 0; k < RB; k++) {
            const int r = r0 + k;
            if (r >= ROWS) continue;
            // the row mask stays in a vector register (the empty asm hides
            // that it is uniform): selects on scalar lane masks would be
            // computed for every pixel up front and spilled
            uint32_t mr = srm[r];
            asm volatile("" : "+v"(mr));
            const float* tp = st + r * RW;
#pragma unroll
            for (int dx = 0; dx < K; dx++) {
                // all ones for a known pixel, zero otherwise: the difference
                // ANDed with it is itself or +0 (NaN included)
                const uint32_t keep = (uint32_t)__builtin_amdgcn_sbfe((int32_t)mr, dx, 1);
#pragma unroll
                for (int ch = 0; ch < C; ch++) {
                    const float dd = tp[dx * C + ch] - vv[k][dx * C + ch];
                    const float d = __uint_as_float(__float_as_uint(dd) & keep);
                    if (NORM == 0) acc = __builtin_fmaf(d, d, acc);
                    else acc = acc + __builtin_fabsf(d);
                }
            }
        }
    }
    return acc;
}

// A handful of queries (the fill loop's lone target, best answer only):
// a query's L*W window entries are split into shares of E <= 64, one
// workgroup each (the share in wave 0), so that a lane costs at most one
// candidate and one query's patch gathers spread over many compute units (a
// single CU's path to L2 would otherwise carry all of them). The workgroup
// has 256 threads only for the apply below. The workgroup stages the
// target and its row masks in LDS, removes the duplicates of its share (LDS
// hash set), costs them (staged_cost), and merges the least (cost, id) into the
// query's packed minimum in global memory (64-bit atomic minimum); the last
// of the query's workgroups to finish, by a ticket counter, writes the
// answer. The packed minimum and the ticket are set to all-ones and zero by
// the prologue. A candidate in two shares is costed twice with the same
// result, so the minimum over the union is unchanged. With apply.ls
// non-null (the fill loop's lone target) that last workgroup also applies
// the answer (apply_pending): every other workgroup has finished reading
// the volume by then.
template <int ND, int K, int C, int NORM>
__global__ __launch_bounds__(256) void rescore_split_kernel(
    QueryIndexView v, const float* vol, const float* __restrict__ t,
    const uint32_t* __restrict__ rowmask, int64_t qpad, const int32_t* __restrict__ qsub,
    const int64_t* __restrict__ wstart, int64_t Q, int P, int E, uint64_t* __restrict__ qbest,
    int32_t* __restrict__ qticket, int64_t* __restrict__ best_id, float* __restrict__ best_cost,
    LoopApply apply) {
    constexpr int ROWS = (ND == 2) ? K : K * K;
    constexpr int NEL = ROWS * K * C;
    constexpr int RB = split_row_group(ND, K, C);
    constexpr int T = 128;   // hash slots: twice the largest share
    __shared__ uint32_t tab[T];
    __shared__ float st[NEL];
    __shared__ uint32_t srm[ROWS];
    const int lane = threadIdx.x;   // the share's entries are all in wave 0 (E <= 64)
    const int64_t q = blockIdx.x / P;
    const int part = (int)(blockIdx.x - q * P);
    if (q >= Q) return;   // uniform: the grid is Q * P workgroups
    const float* tq = t + q * (int64_t)NEL;
    for (int i = lane; i < NEL; i += 64) st[i] = tq[i];
    for (int r = lane; r < ROWS; r += 64) srm[r] = rowmask[(int64_t)r * qpad + q];
    if (lane < T) tab[lane] = 0xffffffffu;
    const int LW = v.L * v.window;
    const int i = part * E + lane;
    uint32_t id = 0xffffffffu;
    if (lane < E && i < LW) {
        const int s = qsub[q];
        const int j = i / v.window, k = i - j * v.window;
        const int64_t pos = wstart[q * v.L + j] + k;
        if (pos < v.n) id = v.ids[((int64_t)s * v.L + j) * v.n + pos];
    }
    __syncthreads();
    uint64_t best = ~0ull;
    if (id != 0xffffffffu) {
        uint32_t h = (id * 0x9E3779B1u) >> (32 - 7);
        bool mine = false;
        while (true) {   // ends: at most 64 of the 128 slots are taken
            const uint32_t old = atomicCAS(&tab[h], 0xffffffffu, id);
            if (old == 0xffffffffu) {
                mine = true;
                break;
            }
            if (old == id) break;
            h = (h + 1) & (uint32_t)(T - 1);
        }
        if (mine) {
            const float cost = staged_cost<ND, K, C, NORM, RB>(v, vol, st, srm, id);
            best = ((uint64_t)__float_as_uint(cost) << 32) | id;
        }
    }
    if (lane < 64) {
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = (uint64_t)__shfl_xor((long long)best, off, 64);
            if (o < best) best = o;
        }
    }
    __shared__ int sh_last;
    int64_t s_ans = -1;
    float c_ans = 0.0f;
    if (lane == 0) {
        if (best != ~0ull) atomicMin(reinterpret_cast<unsigned long long*>(qbest + q), best);
        __threadfence();
        const bool last = atomicAdd(qticket + q, 1) == P - 1;
        if (last) {
            __threadfence();
            // the last workgroup: every other one's minimum is in place
            const uint64_t r = atomicAdd(reinterpret_cast<unsigned long long*>(qbest + q), 0ull);
            s_ans = r == ~0ull ? -1 : (int64_t)(r & 0xffffffffull);
            c_ans = r == ~0ull ? __builtin_inff() : __uint_as_float((uint32_t)(r >> 32));
            best_id[q] = s_ans;
            best_cost[q] = c_ans;
        }
        sh_last = last ? 1 : 0;
    }
    if (!apply.ls) return;
    __syncthreads();
    if (!sh_last) return;   // uniform over the workgroup
    apply_pending(apply, s_ans, c_ans);
}

// One wave per query: exact cost of every listed candidate, (cost, id) min.
template <int ND, int K, int C, int NORM>
__global__ __launch_bounds__(256) void list_rescore_kernel(QueryIndexView v, const float* __restrict__ vol,
                                                           const float* __restrict__ t,
                                                           const uint32_t* __restrict__ rowmask,
                                                           int64_t qpad, const uint32_t* __restrict__ list,
                                                           const int32_t* __restrict__ cnt,
                                                           const int32_t* __restrict__ thr, int cap,
                                                           int64_t Q, int64_t* __restrict__ best_id,
                                                           float* __restrict__ best_cost,
                                                           uint8_t* __restrict__ fb) {
    const int lane = threadIdx.x & 63;
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (q >= Q) return;
    const int nc = cnt[q];
    const bool fallback = thr[q] < 0 || nc > cap || nc == 0;
    if (lane == 0) fb[q] = fallback ? 1 : 0;
    if (fallback) return;
    const float* tq = t + q * (int64_t)v.Kd * C;
    const uint32_t* rm = rowmask + q;
    uint64_t best = ~0ull;
    for (int i = lane; i < nc; i += 64) {
        const uint32_t c = list[q * cap + i];
        const float cost = cand_cost<ND, K, C, NORM>(v, vol, tq, rm, qpad, c);
        const uint64_t pk = ((uint64_t)__float_as_uint(cost) << 32) | c;
        if (pk < best) best = pk;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((long long)best, off, 64);
        if (o < best) best = o;
    }
    if (lane == 0) {
        best_id[q] = (int64_t)(best & 0xffffffffull);
        best_cost[q] = __uint_as_float((uint32_t)(best >> 32));
    }
}

using PrologueFn = void (*)(QueryIndexView, const float*, const uint8_t*, int64_t, int32_t*,
                            double*, uint64_t*, uint32_t*, int64_t);
// ------------------------------------------------------------ exact k-NN
// The k-NN query of Section II.D on the unshifted Morton curve (curve 0 of
// the chosen subset), one wave per query. A region is a box of grid cells
// whose curve interval [a, z) holds exactly the entries whose keys lie
// between the keys of its corners. It is split where the corners first
// differ, at the most significant bit (dimension 0 first among equal
// levels): the low part keeps the upper corner but takes litmax in the split
// dimension (that bit 0, the bits below it 1), the high part keeps the lower
// corner but takes bigmin (that bit 1, the bits below 0). Each part's
// interval comes from a search restricted to the parent's (Section II.E).
// The nearer part is visited first; a part farther from the query cell than
// the k-th nearest entry found so far is skipped. Regions of at most mu
// entries, or of one cell, are scanned: each entry's cell is decoded from
// its key and kept if it ranks among the k smallest (squared distance, id).
// The stack holds only the far parts along the current path, at most
// D*b + 1 frames, in LDS with the k-best list.
constexpr int kKnnMax = 256;   // largest k

struct KnnFrame {
    uint32_t a, z;   // curve interval
    int64_t bd;      // squared distance from the query cell to the box
};

struct KnnArgs {
    QueryIndexView v;
    const int32_t* qsub;
    const double* qcoords;   // [Q][D]
    int64_t Q;
    int k, mu, depth;        // depth: frames of stack space
    uint32_t* list;          // [Q][k] ids of the k nearest, ascending
    int32_t* cnt;            // [Q] entries in list (0 if the query failed)
    int32_t* thr;            // [Q] set to 0 (a valid list for the rescoring)
    unsigned int* overflow;  // set when a stack would overflow
};

__device__ inline bool di_less(int64_t d, uint32_t i, int64_t e, uint32_t j) {
    return d < e || (d == e && i < j);
}

// -1, 0, 1: the key at pos against qk
__device__ inline int key_cmp3(const uint64_t* Kk, int64_t n, int64_t pos, const uint64_t* qk,
                               int W64) {
    for (int w = 0; w < W64; w++) {
        const uint64_t x = Kk[(int64_t)w * n + pos];
        if (x != qk[w]) return x < qk[w] ? -1 : 1;
    }
    return 0;
}

// First position in [a, z) whose key is >= qk (strict: > qk), by rounds of
// 64 probes as in search_kernel; the whole wave calls it.
__device__ int64_t coop_bound(const uint64_t* Kk, int64_t n, int64_t a, int64_t z,
                              const uint64_t* qk, int W64, bool strict, int lane) {
    while (z - a > 64) {
        const int64_t len = z - a;
        const int64_t pos = a + ((int64_t)(lane + 1) * len) / 65;
        const int c = key_cmp3(Kk, n, pos, qk, W64);
        const bool before = strict ? c <= 0 : c < 0;
        const int cnt = __popcll(__ballot(before));
        const int64_t na = cnt > 0 ? a + ((int64_t)cnt * len) / 65 + 1 : a;
        const int64_t nz = cnt < 64 ? a + ((int64_t)(cnt + 1) * len) / 65 : z;
        a = na;
        z = nz;
    }
    bool before = false;
    if (lane < z - a) {
        const int c = key_cmp3(Kk, n, a + lane, qk, W64);
        before = strict ? c <= 0 : c < 0;
    }
    return a + __popcll(__ballot(before));
}

template <int MD>
__device__ inline int64_t box_dist(const uint32_t* lo, const uint32_t* hi, const int64_t* u, int D) {
    int64_t acc = 0;
#pragma unroll
    for (int d = 0; d < MD; d++) {
        if (d < D) {
            int64_t e = 0;
            if (u[d] < (int64_t)lo[d]) e = (int64_t)lo[d] - u[d];
            else if (u[d] > (int64_t)hi[d]) e = u[d] - (int64_t)hi[d];
            acc += e * e;
        }
    }
    return acc;
}

template <int MD>
__global__ __launch_bounds__(64) void knn_kernel(KnnArgs A) {
    extern __shared__ __align__(16) uint8_t knn_smem[];
    const QueryIndexView& v = A.v;
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x;
    if (q >= A.Q) return;
    const int D = v.D, W64 = v.W64, b = v.b, k = A.k;
    const int64_t n = v.n;
    const int s = A.qsub[q];
    const uint64_t* Kk = v.keys + (int64_t)s * v.L * W64 * n;   // curve 0 of subset s
    const uint32_t* ids = v.ids + (int64_t)s * v.L * n;
    int64_t* ldist = reinterpret_cast<int64_t*>(knn_smem);
    uint32_t* lid = reinterpret_cast<uint32_t*>(ldist + kKnnMax);
    KnnFrame* fr = reinterpret_cast<KnnFrame*>(lid + kKnnMax);
    uint32_t* flo = reinterpret_cast<uint32_t*>(fr + A.depth);
    uint32_t* fhi = flo + (int64_t)A.depth * MD;

    // the query's cell on the unshifted curve, by the index query's rule
    int64_t u[MD];
    {
        const double span = (double)v.span[s], rm1 = (double)(v.R - 1);
#pragma unroll
        for (int d = 0; d < MD; d++) {
            u[d] = 0;
            if (d < D) {
                double uu = floor(((A.qcoords[q * D + d] - (double)v.lo[s * D + d]) * rm1) / span);
                if (!(uu >= 0.0)) uu = 0.0;
                if (uu > rm1) uu = rm1;
                u[d] = (int64_t)uu;
            }
        }
    }
    int cntl = 0;                  // entries in the list
    int64_t kd = 0;                // largest (distance, id) of a full list
    uint32_t kid = 0;
    int kpos = 0;
    auto find_max = [&]() {
        int64_t bd = -1;
        uint32_t bi = 0;
        int bp = -1;
        for (int j = lane; j < k; j += 64) {
            const int64_t d = ldist[j];
            const uint32_t i2 = lid[j];
            if (bp < 0 || di_less(bd, bi, d, i2)) {
                bd = d;
                bi = i2;
                bp = j;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const int64_t od = (int64_t)__shfl_xor((long long)bd, off, 64);
            const uint32_t oi = (uint32_t)__shfl_xor((int)bi, off, 64);
            const int op = __shfl_xor(bp, off, 64);
            if (op >= 0 && (bp < 0 || di_less(bd, bi, od, oi))) {
                bd = od;
                bi = oi;
                bp = op;
            }
        }
        kd = bd;
        kid = bi;
        kpos = bp;
    };
    int sp = 0;
    bool overflow = false;
    auto push = [&](uint32_t a, uint32_t z, int64_t bd, const uint32_t* lo, const uint32_t* hi) {
        if (lane == 0) {
            fr[sp] = KnnFrame{a, z, bd};
#pragma unroll
            for (int d = 0; d < MD; d++) {
                flo[sp * MD + d] = lo[d];
                fhi[sp * MD + d] = hi[d];
            }
        }
        sp++;
    };
    {
        uint32_t lo[MD], hi[MD];
#pragma unroll
        for (int d = 0; d < MD; d++) {
            lo[d] = 0;
            hi[d] = d < D ? (uint32_t)(v.R - 1) : 0u;
        }
        push(0u, (uint32_t)n, box_dist<MD>(lo, hi, u, D), lo, hi);
    }
    while (sp > 0) {
        __syncthreads();   // the frame lane 0 wrote is visible
        sp--;
        const KnnFrame f = fr[sp];
        uint32_t lo[MD], hi[MD];
#pragma unroll
        for (int d = 0; d < MD; d++) {
            lo[d] = flo[sp * MD + d];
            hi[d] = fhi[sp * MD + d];
        }
        __syncthreads();   // every lane has read it before it is overwritten
        if (cntl == k && f.bd > kd) continue;
        bool single = true;
#pragma unroll
        for (int d = 0; d < MD; d++)
            if (d < D) single = single && lo[d] == hi[d];
        if ((int64_t)(f.z - f.a) <= A.mu || single) {
            // entries of one cell share their distance and are in id order
            // (the curve is sorted by (key, id)), so only the first k of a
            // one-cell region can rank among the k smallest
            const int64_t zend = single ? min((int64_t)f.z, (int64_t)f.a + k) : (int64_t)f.z;
            for (int64_t base = f.a; base < zend; base += 64) {
                const int64_t i = base + lane;
                const bool live = i < zend;
                int64_t dist = 0;
                uint32_t id = 0;
                if (live) {
                    uint64_t w[kMaxKeyWords];
#pragma unroll
                    for (int j = 0; j < kMaxKeyWords; j++) w[j] = j < W64 ? Kk[(int64_t)j * n + i] : 0ull;
                    uint32_t c[MD];
                    morton_decode<MD>(w, D, b, W64, c);
#pragma unroll
                    for (int d = 0; d < MD; d++) {
                        if (d < D) {
                            const int64_t e = (int64_t)c[d] - u[d];
                            dist += e * e;
                        }
                    }
                    id = ids[i];
                }
                uint64_t mask = __ballot(live && (cntl < k || di_less(dist, id, kd, kid)));
                while (mask) {
                    const int src = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const int64_t dd = (int64_t)__shfl((long long)dist, src, 64);
                    const uint32_t ii = (uint32_t)__shfl((int)id, src, 64);
                    if (cntl < k) {
                        if (lane == 0) {
                            ldist[cntl] = dd;
                            lid[cntl] = ii;
                        }
                        cntl++;
                        if (cntl == k) {
                            __syncthreads();
                            find_max();
                        }
                    } else if (di_less(dd, ii, kd, kid)) {
                        if (lane == 0) {
                            ldist[kpos] = dd;
                            lid[kpos] = ii;
                        }
                        __syncthreads();
                        find_max();
                    }
                }
            }
            continue;
        }
        // split at the most significant differing bit
        int sd = 0, sh = -1;
#pragma unroll
        for (int d = 0; d < MD; d++) {
            if (d < D) {
                const uint32_t x = lo[d] ^ hi[d];
                if (x) {
                    const int h = 31 - __builtin_clz(x);
                    if (h > sh) {
                        sh = h;
                        sd = d;
                    }
                }
            }
        }
        uint32_t lit[MD], big[MD];
#pragma unroll
        for (int d = 0; d < MD; d++) {
            lit[d] = hi[d];
            big[d] = lo[d];
        }
        uint32_t hs = 0, ls = 0;
#pragma unroll
        for (int d = 0; d < MD; d++)
            if (d == sd) hs = hi[d];
        const uint32_t pre = (uint32_t)(((uint64_t)hs >> (sh + 1)) << (sh + 1));
        ls = pre | ((1u << sh) - 1u);
        hs = pre | (1u << sh);
#pragma unroll
        for (int d = 0; d < MD; d++) {
            if (d == sd) {
                lit[d] = ls;
                big[d] = hs;
            }
        }
        uint64_t kl[kMaxKeyWords], kb[kMaxKeyWords];
        interleave_words<MD>(lit, D, b, W64, kl);
        interleave_words<MD>(big, D, b, W64, kb);
        const int64_t zl = coop_bound(Kk, n, f.a, f.z, kl, W64, true, lane);
        const int64_t ah = coop_bound(Kk, n, zl, f.z, kb, W64, false, lane);
        const int64_t bl = box_dist<MD>(lo, lit, u, D), bh = box_dist<MD>(big, hi, u, D);
        const bool use_l = f.a < zl && !(cntl == k && bl > kd);
        const bool use_h = ah < f.z && !(cntl == k && bh > kd);
        if (sp + 2 > A.depth) {
            overflow = true;
            break;
        }
        // the far part first, so that the near one is popped next
        if (bl <= bh) {
            if (use_h) push((uint32_t)ah, f.z, bh, big, hi);
            if (use_l) push(f.a, (uint32_t)zl, bl, lo, lit);
        } else {
            if (use_l) push(f.a, (uint32_t)zl, bl, lo, lit);
            if (use_h) push((uint32_t)ah, f.z, bh, big, hi);
        }
    }
    __syncthreads();
    if (overflow) {
        if (lane == 0) {
            A.cnt[q] = 0;
            A.thr[q] = 0;
            atomicOr(A.overflow, 1u);
        }
        return;
    }
    // ascending ids (they are distinct: every entry is visited at most once)
    for (int j = lane; j < cntl; j += 64) {
        const uint32_t x = lid[j];
        int r = 0;
        for (int t2 = 0; t2 < cntl; t2++) r += lid[t2] < x ? 1 : 0;
        A.list[q * k + r] = x;
    }
    if (lane == 0) {
        A.cnt[q] = cntl;
        A.thr[q] = 0;
    }
}

__global__ void knn_cand_kernel(const uint32_t* __restrict__ list, const int32_t* __restrict__ cnt,
                                int64_t Q, int k, int64_t* __restrict__ cand,
                                int32_t* __restrict__ ncand) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q * k) return;
    const int64_t q = i / k;
    const int j = (int)(i - q * k);
    if (cand) cand[i] = j < cnt[q] ? (int64_t)list[i] : -1;
    if (ncand && j == 0) ncand[q] = cnt[q];
}

using RescoreFn = void (*)(QueryIndexView, const float*, const float*, const uint32_t*, int64_t,
                           const int32_t*, const int64_t*, int64_t, int, int64_t*, float*,
                           int64_t*, int32_t*, int);

using PrologueOneFn = void (*)(QueryIndexView, const float*, const uint8_t*, int64_t, int32_t*,
                               double*, uint64_t*, uint32_t*, int64_t, uint64_t*, int32_t*);
struct PrologueEntry {
    PrologueFn many;
    PrologueOneFn one;
};
template <int D>
PrologueEntry prologue_entry() {
    return {prologue_kernel<D, kPrologueLanes>, prologue_one_kernel<D>};
}

using ListFn = void (*)(QueryIndexView, const float*, const float*, const uint32_t*, int64_t,
                       const uint32_t*, const int32_t*, const int32_t*, int, int64_t, int64_t*,
                       float*, uint8_t*);

// fn / fn_l1: large batches (one row of a candidate per memory round
// trip, few registers); gfn / gfn_l1: up to kRescoreSharedQ queries (rows
// requested in groups, for the latency of small batches)
using SplitFn = void (*)(QueryIndexView, const float*, const float*, const uint32_t*, int64_t,
                         const int32_t*, const int64_t*, int64_t, int, int, uint64_t*, int32_t*,
                         int64_t*, float*, LoopApply);
struct RescoreEntry {
    int nd, K, C;
    RescoreFn fn, fn_l1, gfn, gfn_l1;
    ListFn lfn, lfn_l1;
    SplitFn sfn, sfn_l1;
};
#define SFC_RESCORE(ND, K, C)                                                                 \
    {ND, K, C, rescore_kernel<ND, K, C, 0>, rescore_kernel<ND, K, C, 1>,                     \
     rescore_kernel<ND, K, C, 0, cost_row_group(ND, K, C)>,                                 \
     rescore_kernel<ND, K, C, 1, cost_row_group(ND, K, C)>,                                 \
     list_rescore_kernel<ND, K, C, 0>, list_rescore_kernel<ND, K, C, 1>,                    \
     rescore_split_kernel<ND, K, C, 0>, rescore_split_kernel<ND, K, C, 1>}
const RescoreEntry kRescore[] = {
    SFC_RESCORE(2, 3, 1), SFC_RESCORE(2, 3, 2), SFC_RESCORE(2, 3, 3),
    SFC_RESCORE(2, 5, 1), SFC_RESCORE(2, 5, 2), SFC_RESCORE(2, 5, 3),
    SFC_RESCORE(2, 7, 1), SFC_RESCORE(2, 7, 2), SFC_RESCORE(2, 7, 3),
    SFC_RESCORE(2, 9, 1), SFC_RESCORE(2, 9, 2), SFC_RESCORE(2, 9, 3),
    SFC_RESCORE(2, 11, 1), SFC_RESCORE(2, 11, 3),
    SFC_RESCORE(2, 13, 1), SFC_RESCORE(2, 13, 3),
    SFC_RESCORE(3, 3, 1), SFC_RESCORE(3, 3, 2),
    SFC_RESCORE(3, 5, 1), SFC_RESCORE(3, 5, 2),
    SFC_RESCORE(3, 7, 1),
};

}  // namespace

sfc_status launch_query_prologue(const QueryIndexView& v, const float* t, const uint8_t* m,
                                 int64_t Q, int32_t* qsub, double* qcoords, uint64_t* qkeys,
                                 uint32_t* rowmask, int64_t qpad, uint64_t* qbest,
                                 int32_t* qticket, hipStream_t st) {
    if (Q == 0) return SFC_OK;
    PrologueEntry fn{};
    switch (v.D) {
    case 1: fn = prologue_entry<1>(); break;
    case 2: fn = prologue_entry<2>(); break;
    case 3: fn = prologue_entry<3>(); break;
    case 4: fn = prologue_entry<4>(); break;
    case 5: fn = prologue_entry<5>(); break;
    case 6: fn = prologue_entry<6>(); break;
    case 7: fn = prologue_entry<7>(); break;
    case 8: fn = prologue_entry<8>(); break;
    case 9: fn = prologue_entry<9>(); break;
    case 10: fn = prologue_entry<10>(); break;
    case 11: fn = prologue_entry<11>(); break;
    case 12: fn = prologue_entry<12>(); break;
    case 16: fn = prologue_entry<16>(); break;
    default: return fail(SFC_EUNSUPPORTED, "index query: reduced dimension not in {1..12, 16}");
    }
    if (v.Kd > 64 * kMaxKnownWords || v.S > kMaxSubsets)
        return fail(SFC_EUNSUPPORTED, "index query: more than 1024 pixels or 26 subsets per patch");
    if ((qbest == nullptr) != (qticket == nullptr))
        return fail(SFC_EINVAL, "index query: packed best and ticket go together");
    // few queries: a workgroup per query, whose loads go out phase by phase
    // (the split rescoring, for at most kRescoreSplitQ <= kPrologueWideQ
    // queries, relies on this kernel to clear its words)
    if (Q <= kPrologueWideQ) {
        hipLaunchKernelGGL(fn.one, dim3((unsigned)Q), dim3(256), 0, st, v, t, m, Q, qsub, qcoords,
                           qkeys, rowmask, qpad, qbest, qticket);
        return launched("prologue_one_kernel");
    }
    hipLaunchKernelGGL(fn.many, dim3(blocks_for(Q, 256 / kPrologueLanes)), dim3(256), 0, st, v, t,
                       m, Q, qsub, qcoords, qkeys, rowmask, qpad);
    return launched("prologue_kernel");
}

sfc_status launch_query_search(const QueryIndexView& v, const int32_t* qsub, const uint64_t* qkeys,
                               int64_t Q, int64_t* wstart, hipStream_t st) {
    if (Q == 0) return SFC_OK;
    // up to a few thousand searches: one wave each; beyond, four per wave
    if (Q * v.L <= 4096)
        search_kernel<64><<<blocks_for(Q * v.L * 64), 256, 0, st>>>(v, qsub, qkeys, Q, wstart);
    else
        search_kernel<16><<<blocks_for(Q * v.L * 16), 256, 0, st>>>(v, qsub, qkeys, Q, wstart);
    return launched("search_kernel");
}

sfc_status launch_list_rescore(const Grid& g, const float* vol, const float* t,
                               const uint32_t* rowmask, int64_t qpad, const uint32_t* list,
                               const int32_t* cnt, const int32_t* thr, int cap, int64_t Q,
                               int64_t* best_id, float* best_cost, uint8_t* fb, int norm,
                               hipStream_t st) {
    if (Q == 0) return SFC_OK;
    const RescoreEntry* ent = nullptr;
    for (const auto& e : kRescore)
        if (e.nd == g.nd && e.K == g.K && e.C == g.C) ent = &e;
    if (!ent) return fail(SFC_EUNSUPPORTED, "list rescoring: no kernel for this (ndim, K, C)");
    QueryIndexView v{};
    v.nd = g.nd;
    v.K = g.K;
    v.C = g.C;
    v.Kd = g.Kd;
    for (int i = 0; i < kMaxDims; i++) {
        v.shape[i] = g.shape[i];
        v.stride[i] = g.stride[i];
    }
    hipLaunchKernelGGL(norm == 1 ? ent->lfn_l1 : ent->lfn, dim3(blocks_for(Q * 64)), dim3(256), 0,
                       st, v, vol, t, rowmask, qpad, list, cnt, thr, cap, Q, best_id, best_cost, fb);
    return launched("list_rescore_kernel");
}

bool rescore_supported(int nd, int K, int C) {
    for (const auto& e : kRescore)
        if (e.nd == nd && e.K == K && e.C == C) return true;
    return false;
}

sfc_status launch_query_rescore(const QueryIndexView& v, const float* vol, const float* t,
                                const uint32_t* rowmask, int64_t qpad, const int32_t* qsub,
                                const int64_t* wstart, int64_t Q, int64_t* best_id,
                                float* best_cost, int64_t* cand, int32_t* ncand, int norm,
                                uint64_t* qbest, int32_t* qticket, const LoopApply* apply,
                                hipStream_t st) {
    if (Q == 0) return SFC_OK;
    const RescoreEntry* ent = nullptr;
    for (const auto& e : kRescore)
        if (e.nd == v.nd && e.K == v.K && e.C == v.C) ent = &e;
    if (!ent) return fail(SFC_EUNSUPPORTED, "index rescoring: no kernel for this (ndim, K, C)");
    int cap = 64;
    while (cap < v.L * v.window) cap <<= 1;
    if (cap > kCap) return fail(SFC_EUNSUPPORTED, "n_curves * window above 2048");
    // a handful of queries, best answer only: each query's windows split
    // over workgroups (the prologue cleared the packed minima and tickets)
    if (Q <= kRescoreSplitQ && !cand && !ncand && best_id && best_cost && qbest && qticket) {
        // shares of E entries (a power of two, 8..64) whose patches hold
        // about kSplitShareBytes
        const int64_t patch = (int64_t)v.Kd * v.C * 4;
        int E = 64;
        while (E > 8 && E * patch > kSplitShareBytes) E >>= 1;
        const int P = (v.L * v.window + E - 1) / E;
        LoopApply la{};
        if (apply) {
            if (Q != 1) return fail(SFC_EINVAL, "index rescoring: the loop's apply takes one query");
            la = *apply;
        }
        hipLaunchKernelGGL(norm == 1 ? ent->sfn_l1 : ent->sfn, dim3((unsigned)(Q * P)), dim3(256),
                           0, st, v, vol, t, rowmask, qpad, qsub, wstart, Q, P, E, qbest, qticket,
                           best_id, best_cost, la);
        return launched("rescore_split_kernel");
    }
    if (apply) return fail(SFC_EUNSUPPORTED, "index rescoring: the loop's apply needs the split form");
    const size_t lds = (size_t)8 * cap * sizeof(uint32_t);
    // few queries: a workgroup per query (four waves split its candidates)
    // and candidate rows requested in groups; a multiple of 8 workgroups, so
    // the XCD-aware query order is a bijection
    const bool few = Q <= kRescoreSharedQ;
    const int wpq = few ? 4 : 1;
    const RescoreFn kfn = few ? (norm == 1 ? ent->gfn_l1 : ent->gfn) : (norm == 1 ? ent->fn_l1 : ent->fn);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return check_hip(e, "rescore LDS attribute");
    }
    const unsigned nblk = (blocks_for(Q, 4 / wpq) + 7) / 8 * 8;
    hipLaunchKernelGGL(kfn, dim3(nblk), dim3(256), lds,
                       st, v, vol, t, rowmask, qpad, qsub, wstart, Q, cap, best_id, best_cost,
                       cand, ncand, wpq);
    return launched("rescore_kernel");
}

sfc_status launch_knn(const QueryIndexView& v, const int32_t* qsub, const double* qcoords,
                      int64_t Q, int k, int mu, uint32_t* list, int32_t* cnt, int32_t* thr,
                      unsigned int* overflow, hipStream_t st) {
    if (Q == 0) return SFC_OK;
    if (k < 1 || k > kKnnMax) return fail(SFC_EINVAL, "k-NN query: k must be 1..256");
    if (v.D < 1 || v.D > 16) return fail(SFC_EUNSUPPORTED, "k-NN query: reduced dimension above 16");
    const int md = v.D <= 8 ? 8 : 16;
    KnnArgs A{};
    A.v = v;
    A.qsub = qsub;
    A.qcoords = qcoords;
    A.Q = Q;
    A.k = k;
    A.mu = mu;
    A.depth = v.D * v.b + 2;
    A.list = list;
    A.cnt = cnt;
    A.thr = thr;
    A.overflow = overflow;
    const size_t lds = (size_t)kKnnMax * 12 + (size_t)A.depth * (sizeof(KnnFrame) + 8 * md);
    if (lds > 160 * 1024) return fail(SFC_EUNSUPPORTED, "k-NN query: D * key_bits too large");
    const void* fn = md == 8 ? (const void*)knn_kernel<8> : (const void*)knn_kernel<16>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return check_hip(e, "k-NN LDS attribute");
    }
    if (Q > 0x7fffffffLL) return fail(SFC_EUNSUPPORTED, "k-NN query: too many queries");
    if (md == 8) knn_kernel<8><<<(unsigned)Q, 64, lds, st>>>(A);
    else knn_kernel<16><<<(unsigned)Q, 64, lds, st>>>(A);
    return launched("knn_kernel");
}

sfc_status launch_knn_cand(const uint32_t* list, const int32_t* cnt, int64_t Q, int k,
                           int64_t* cand, int32_t* ncand, hipStream_t st) {
    if (Q == 0 || (!cand && !ncand)) return SFC_OK;
    knn_cand_kernel<<<blocks_for(Q * k), 256, 0, st>>>(list, cnt, Q, k, cand, ncand);
    return launched("knn_cand_kernel");
}

}  // namespace sfc
