// Index query (Fig. 1 b-d): choose the subset index that best covers the
// known pixels of the target, move the query to principal space, find its
// position on each shifted curve by a wave-cooperative search, take a window
// of entries around it per curve, and rescore the union of the windows with
// the exact masked cost (a full scan in image space over the candidates).
#include "keys.hpp"
#include "mfma_scan.hpp"
#include "query.hpp"

namespace sfc {

namespace {

typedef const __attribute__((address_space(4))) float cfloat_as4;
typedef const __attribute__((address_space(4))) uint32_t cu32_as4;
__device__ inline float ldu(const float* p) { return *(cfloat_as4*)p; }
__device__ inline uint32_t ldu(const uint32_t* p) { return *(cu32_as4*)p; }

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}

// ------------------------------------------------------------ prologue
// One thread per query. Subset: the largest known fraction k_s/n_s, compared
// exactly as k_a*n_b > k_b*n_a, ties to the lower subset. Coordinates: the
// known elements enter exactly (A = W_k^T x_k); unknown ones are imputed from
// the principal-component model fitted to the known ones by least squares:
//   G = W^T W - W_u^T W_u + I,  r = W_k^T (n_sub x_k - S_k)   (integers)
//   G z = r by Gaussian elimination without pivoting (float64, column by
//   column, then back substitution),
//   y_d = A_d + (B_d + sum_e H_de z_e) / n_sub,  B = W_u^T S_u,  H = W_u^T W_u.
template <int D>
__global__ __launch_bounds__(64) void prologue_kernel(QueryIndexView v, const float* __restrict__ t,
                                                      const uint8_t* __restrict__ m, int64_t Q,
                                                      int32_t* __restrict__ qsub,
                                                      double* __restrict__ qcoords,
                                                      uint64_t* __restrict__ qkeys) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const uint8_t* mq = m + q * v.Kd;
    const float* tq = t + q * v.Kd * v.C;
    int sb = 0;
    int64_t kb = -1, nbest = 1;
    for (int s = 0; s < v.S; s++) {
        const int ns = v.npix[s];
        int64_t k = 0;
        for (int i = 0; i < ns; i++) k += mq[v.pix[s * v.Kd + i]] ? 1 : 0;
        if (kb < 0 || k * nbest > kb * ns) {
            sb = s;
            kb = k;
            nbest = ns;
        }
    }
    const float vmin = v.qparams[0], sc = v.qparams[1];
    int64_t A[D], B[D], r[D], H[D][D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        A[d] = 0;
        B[d] = 0;
        r[d] = 0;
#pragma unroll
        for (int f = 0; f < D; f++) H[d][f] = 0;
    }
    const int8_t* wb = v.basis + (int64_t)sb * v.mmax * D;
    int row = 0;
    for (int i = 0; i < v.npix[sb]; i++) {
        const int rho = v.pix[sb * v.Kd + i];
        const bool known = mq[rho] != 0;
        for (int ch = 0; ch < v.C; ch++, row++) {
            const int e = rho * v.C + ch;
            int64_t w[D];
#pragma unroll
            for (int d = 0; d < D; d++) w[d] = wb[row * D + d];
            if (known) {
                float rr = __builtin_rintf((tq[e] - vmin) * sc);
                if (!(rr >= 0.0f)) rr = 0.0f;
                if (rr > 255.0f) rr = 255.0f;
                const int64_t x = (int64_t)rr;
                const int64_t c = v.nsub * x - (int64_t)v.sum[e];
#pragma unroll
                for (int d = 0; d < D; d++) {
                    A[d] += w[d] * x;
                    r[d] += w[d] * c;
                }
            } else {
                const int64_t se = (int64_t)v.sum[e];
#pragma unroll
                for (int d = 0; d < D; d++) {
                    B[d] += w[d] * se;
#pragma unroll
                    for (int f = 0; f < D; f++) H[d][f] += w[d] * w[f];
                }
            }
        }
    }
    const int64_t* wtw = v.wtw + (int64_t)sb * D * D;
    double a[D][D], rr[D], z[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
#pragma unroll
        for (int f = 0; f < D; f++) a[d][f] = (double)(wtw[d * D + f] - H[d][f] + (d == f ? 1 : 0));
        rr[d] = (double)r[d];
    }
#pragma unroll
    for (int k = 0; k < D; k++)
#pragma unroll
        for (int i = k + 1; i < D; i++) {
            const double fct = a[i][k] / a[k][k];
#pragma unroll
            for (int j = k + 1; j < D; j++) a[i][j] = a[i][j] - fct * a[k][j];
            rr[i] = rr[i] - fct * rr[k];
        }
#pragma unroll
    for (int i = D - 1; i >= 0; i--) {
        double s = rr[i];
#pragma unroll
        for (int j = i + 1; j < D; j++) s = s - a[i][j] * z[j];
        z[i] = s / a[i][i];
    }
    double y[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        double f = (double)B[d];
#pragma unroll
        for (int e = 0; e < D; e++) f = f + (double)H[d][e] * z[e];
        y[d] = (double)A[d] + f / (double)v.nsub;
        qcoords[q * D + d] = y[d];
    }
    qsub[q] = sb;
    // grid cell and one key per shifted curve
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
    for (int j = 0; j < v.L; j++) {
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
__device__ inline bool key_less(const uint64_t* K, int64_t n, int64_t pos, const uint64_t* qk,
                                int W64) {
    for (int w = 0; w < W64; w++) {
        const uint64_t a = K[(int64_t)w * n + pos];
        if (a != qk[w]) return a < qk[w];
    }
    return false;
}

// One wave per (query, curve): first position whose key is >= the query key,
// by rounds of 64 probes splitting the interval into 65 parts (ballot gives
// the number of probes below the key), then a final round over <= 64 entries.
__global__ __launch_bounds__(256) void search_kernel(QueryIndexView v, const int32_t* __restrict__ qsub,
                                                     const uint64_t* __restrict__ qkeys, int64_t Q,
                                                     int64_t* __restrict__ wstart) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wid >= Q * v.L) return;
    const int64_t q = wid / v.L;
    const int j = (int)(wid - q * v.L);
    const int s = qsub[q];
    const uint64_t* K = v.keys + ((int64_t)s * v.L + j) * v.W64 * v.n;
    uint64_t qk[kMaxKeyWords];
    for (int w = 0; w < v.W64; w++) qk[w] = qkeys[(q * v.L + j) * v.W64 + w];
    int64_t a = 0, z = v.n;
    while (z - a > 64) {
        const int64_t len = z - a;
        const int64_t pos = a + ((int64_t)(lane + 1) * len) / 65;
        const bool less = key_less(K, v.n, pos, qk, v.W64);
        const int cnt = __popcll(__ballot(less));
        const int64_t na = cnt > 0 ? a + ((int64_t)cnt * len) / 65 + 1 : a;
        const int64_t nz = cnt < 64 ? a + ((int64_t)(cnt + 1) * len) / 65 : z;
        a = na;
        z = nz;
    }
    const int64_t len = z - a;
    const bool less = lane < len && key_less(K, v.n, a + lane, qk, v.W64);
    const int64_t p = a + __popcll(__ballot(less));
    int64_t lo = p - v.window / 2;
    int64_t lmax = v.n - v.window;
    if (lmax < 0) lmax = 0;
    if (lo > lmax) lo = lmax;
    if (lo < 0) lo = 0;
    if (lane == 0) wstart[wid] = lo;
}

// ------------------------------------------------------------ rescore
constexpr int kCap = 512;   // maximum L*W

template <int ND, int K, int C, int NORM>
__device__ inline float cand_cost(const QueryIndexView& v, const float* __restrict__ vol,
                                  const float* __restrict__ tq, const uint32_t* __restrict__ rm,
                                  int64_t qpad, uint32_t c) {
    constexpr int H = (K - 1) / 2;
    constexpr int ROWS = (ND == 2) ? K : K * K;
    constexpr int RW = K * C;
    float acc = 0.0f;
    for (int r = 0; r < ROWS; r++) {
        const uint32_t mr = ldu(rm + (int64_t)r * qpad);
        if (mr == 0) continue;
        int64_t roff;
        if (ND == 2) roff = (int64_t)(r - H) * v.stride[0] - H;
        else roff = (int64_t)(r / K - H) * v.stride[0] + (int64_t)(r % K - H) * v.stride[1] - H;
        const float* vp = vol + ((int64_t)c + roff) * C;
        float vv[RW];
#pragma unroll
        for (int i = 0; i < RW; i++) vv[i] = vp[i];
        const float* tp = tq + (int64_t)r * RW;
#pragma unroll
        for (int dx = 0; dx < K; dx++) {
            if (mr & (1u << dx)) {
#pragma unroll
                for (int ch = 0; ch < C; ch++) {
                    const float d = ldu(tp + dx * C + ch) - vv[dx * C + ch];
                    // d*d fused (L2) or |d| added (L1, Section III.K)
                    if (NORM == 0) acc = __builtin_fmaf(d, d, acc);
                    else acc = acc + __builtin_fabsf(d);
                }
            }
        }
    }
    return acc;
}

// One wave per query: gather the window ids, sort them in LDS (bitonic),
// keep the unique ones, then each lane rescores every 64th candidate.
template <int ND, int K, int C, int NORM>
__global__ __launch_bounds__(256) void rescore_kernel(QueryIndexView v, const float* __restrict__ vol,
                                                      const float* __restrict__ t,
                                                      const uint32_t* __restrict__ rowmask,
                                                      int64_t qpad, const int32_t* __restrict__ qsub,
                                                      const int64_t* __restrict__ wstart, int64_t Q,
                                                      int cap, int64_t* __restrict__ best_id,
                                                      float* __restrict__ best_cost,
                                                      int64_t* __restrict__ cand,
                                                      int32_t* __restrict__ ncand) {
    __shared__ uint32_t sa[4][kCap];
    __shared__ uint32_t sb[4][kCap];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * 4 + w;
    const bool live = q < Q;
    const int LW = v.L * v.window;
    uint32_t* A = sa[w];
    uint32_t* Bu = sb[w];
    const int s = live ? qsub[q] : 0;
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
    if (!live) return;
    if (cand) {
        for (int i = lane; i < LW; i += 64) cand[q * LW + i] = i < nu ? (int64_t)Bu[i] : -1;
        if (lane == 0) ncand[q] = nu;
    }
    if (!best_id) return;
    const float* tq = t + q * (int64_t)v.Kd * C;
    const uint32_t* rm = rowmask + q;
    uint64_t best = ~0ull;
    for (int i = lane; i < nu; i += 64) {
        const uint32_t c = Bu[i];
        const float cost = cand_cost<ND, K, C, NORM>(v, vol, tq, rm, qpad, c);
        const uint64_t pk = ((uint64_t)__float_as_uint(cost) << 32) | c;
        if (pk < best) best = pk;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((long long)best, off, 64);
        if (o < best) best = o;
    }
    if (lane == 0) {
        best_id[q] = best == ~0ull ? -1 : (int64_t)(best & 0xffffffffull);
        best_cost[q] = best == ~0ull ? __builtin_inff() : __uint_as_float((uint32_t)(best >> 32));
    }
}

// One wave per query: exact cost of every listed candidate, (cost, id) min.
template <int ND, int K, int C>
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
        const float cost = cand_cost<ND, K, C, 0>(v, vol, tq, rm, qpad, c);
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
                            double*, uint64_t*);
using RescoreFn = void (*)(QueryIndexView, const float*, const float*, const uint32_t*, int64_t,
                           const int32_t*, const int64_t*, int64_t, int, int64_t*, float*,
                           int64_t*, int32_t*);

template <int D>
PrologueFn prologue_fn() { return prologue_kernel<D>; }

using ListFn = void (*)(QueryIndexView, const float*, const float*, const uint32_t*, int64_t,
                       const uint32_t*, const int32_t*, const int32_t*, int, int64_t, int64_t*,
                       float*, uint8_t*);

struct RescoreEntry {
    int nd, K, C;
    RescoreFn fn, fn_l1;
    ListFn lfn;
};
#define SFC_RESCORE(ND, K, C)                                                                 \
    {ND, K, C, rescore_kernel<ND, K, C, 0>, rescore_kernel<ND, K, C, 1>, list_rescore_kernel<ND, K, C>}
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
                                 hipStream_t st) {
    if (Q == 0) return SFC_OK;
    PrologueFn fn = nullptr;
    switch (v.D) {
    case 1: fn = prologue_fn<1>(); break;
    case 2: fn = prologue_fn<2>(); break;
    case 3: fn = prologue_fn<3>(); break;
    case 4: fn = prologue_fn<4>(); break;
    case 5: fn = prologue_fn<5>(); break;
    case 6: fn = prologue_fn<6>(); break;
    case 7: fn = prologue_fn<7>(); break;
    case 8: fn = prologue_fn<8>(); break;
    case 9: fn = prologue_fn<9>(); break;
    case 10: fn = prologue_fn<10>(); break;
    case 11: fn = prologue_fn<11>(); break;
    case 12: fn = prologue_fn<12>(); break;
    case 16: fn = prologue_fn<16>(); break;
    default: return fail(SFC_EUNSUPPORTED, "index query: reduced dimension not in {1..12, 16}");
    }
    hipLaunchKernelGGL(fn, dim3(blocks_for(Q, 64)), dim3(64), 0, st, v, t, m, Q, qsub, qcoords,
                       qkeys);
    return launched("prologue_kernel");
}

sfc_status launch_query_search(const QueryIndexView& v, const int32_t* qsub, const uint64_t* qkeys,
                               int64_t Q, int64_t* wstart, hipStream_t st) {
    if (Q == 0) return SFC_OK;
    search_kernel<<<blocks_for(Q * v.L * 64), 256, 0, st>>>(v, qsub, qkeys, Q, wstart);
    return launched("search_kernel");
}

sfc_status launch_list_rescore(const Grid& g, const float* vol, const float* t,
                               const uint32_t* rowmask, int64_t qpad, const uint32_t* list,
                               const int32_t* cnt, const int32_t* thr, int cap, int64_t Q,
                               int64_t* best_id, float* best_cost, uint8_t* fb, hipStream_t st) {
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
    hipLaunchKernelGGL(ent->lfn, dim3(blocks_for(Q * 64)), dim3(256), 0, st, v, vol, t, rowmask,
                       qpad, list, cnt, thr, cap, Q, best_id, best_cost, fb);
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
                                hipStream_t st) {
    if (Q == 0) return SFC_OK;
    const RescoreEntry* ent = nullptr;
    for (const auto& e : kRescore)
        if (e.nd == v.nd && e.K == v.K && e.C == v.C) ent = &e;
    if (!ent) return fail(SFC_EUNSUPPORTED, "index rescoring: no kernel for this (ndim, K, C)");
    int cap = 64;
    while (cap < v.L * v.window) cap <<= 1;
    if (cap > kCap) return fail(SFC_EUNSUPPORTED, "n_curves * window above 512");
    hipLaunchKernelGGL(norm == 1 ? ent->fn_l1 : ent->fn, dim3(blocks_for(Q, 4)), dim3(256), 0, st,
                       v, vol, t, rowmask, qpad, qsub, wstart, Q, cap, best_id, best_cost, cand,
                       ncand);
    return launched("rescore_kernel");
}

}  // namespace sfc
