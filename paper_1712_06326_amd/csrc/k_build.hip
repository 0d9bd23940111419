// Index build, part 1 (Sections II, II.A): byte quantisation of the volume,
// exact integer patch statistics over a strided subsample of the dictionary,
// per-subset covariance, float64 Jacobi eigendecomposition and the int8
// basis of the first D principal components.
#include "build.hpp"

namespace sfc {

namespace {

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}

// ------------------------------------------------------------ quantisation
// Order-preserving unsigned encoding of a float (for atomic min/max).
__device__ inline uint32_t fenc(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float fdec(uint32_t e) {
    return __uint_as_float((e & 0x80000000u) ? (e & 0x7fffffffu) : ~e);
}

__global__ void minmax_init_kernel(uint32_t* mm) {
    mm[0] = 0xffffffffu;
    mm[1] = 0u;
}

__global__ void minmax_kernel(const float* __restrict__ vol, const uint8_t* __restrict__ mask,
                              int64_t nvox, int C, uint32_t* __restrict__ mm) {
    uint32_t lo = 0xffffffffu, hi = 0u;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (!mask[v]) continue;
        for (int ch = 0; ch < C; ch++) {
            const uint32_t e = fenc(vol[v * C + ch]);
            lo = min(lo, e);
            hi = max(hi, e);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}

// params = {vmin, scale = 255 / (vmax - vmin) in float32 (0 when the range is
// empty), vmax}
__global__ void scale_kernel(const uint32_t* __restrict__ mm, float* __restrict__ params) {
    const float lo = fdec(mm[0]), hi = fdec(mm[1]);
    params[0] = lo;
    params[1] = (hi > lo) ? 255.0f / (hi - lo) : 0.0f;
    params[2] = hi;
}

__global__ void quantize_kernel(const float* __restrict__ vol, int64_t n,
                                const float* __restrict__ params, uint8_t* __restrict__ xq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float lo = params[0], s = params[1];
    float r = __builtin_rintf((vol[i] - lo) * s);
    if (!(r >= 0.0f)) r = 0.0f;
    if (r > 255.0f) r = 255.0f;
    xq[i] = (uint8_t)r;
}

// ------------------------------------------------------------ covariance
// Xt[e][s4] packs the bytes of samples 4*s4 .. 4*s4+3 of element e.
__global__ void gather_samples_kernel(const uint8_t* __restrict__ xq,
                                      const uint32_t* __restrict__ dict, int64_t stride,
                                      int64_t nsub, const int32_t* __restrict__ elem_off, int P,
                                      int C, uint32_t* __restrict__ Xt, int64_t nsp4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)P * nsp4) return;
    const int e = (int)(i / nsp4);
    const int64_t s4 = i - (int64_t)e * nsp4;
    const int64_t off = elem_off[e];
    uint32_t w = 0;
    for (int k = 0; k < 4; k++) {
        const int64_t s = s4 * 4 + k;
        if (s < nsub) {
            const int64_t c = dict[s * stride];
            w |= (uint32_t)xq[c * C + off] << (8 * k);
        }
    }
    Xt[i] = w;
}

// sum[e] = sum of all sample bytes of element e (one block per element)
__global__ void sample_sum_kernel(const uint32_t* __restrict__ Xt, int64_t nsp4,
                                  uint64_t* __restrict__ sum) {
    const int e = blockIdx.x;
    uint64_t acc = 0;
    for (int64_t k = threadIdx.x; k < nsp4; k += blockDim.x) {
        const uint32_t w = Xt[(int64_t)e * nsp4 + k];
        acc += (w & 0xff) + ((w >> 8) & 0xff) + ((w >> 16) & 0xff) + (w >> 24);
    }
    __shared__ uint64_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sum[e] = red[0];
}

constexpr int kGT = 64;        // gram tile (elements)
constexpr int kGK = 32;        // dwords per LDS stage
constexpr int kGChunk = 4096;  // dwords (16384 samples) per block: u32 partials cannot overflow

// gram[e][f] += sum over samples of x_e * x_f, for tiles E <= F, with
// v_dot4_u32_u8 on 4 packed samples at a time.
__global__ __launch_bounds__(256) void gram_kernel(const uint32_t* __restrict__ Xt, int P,
                                                   int64_t nsp4, int ntiles,
                                                   uint64_t* __restrict__ gram) {
    // decode the (E, F) upper-triangular tile pair
    int pair = blockIdx.x, E = 0;
    while (pair >= ntiles - E) {
        pair -= ntiles - E;
        E++;
    }
    const int F = E + pair;
    const int64_t k0 = (int64_t)blockIdx.y * kGChunk;
    const int64_t k1 = min(nsp4, k0 + kGChunk);
    __shared__ uint32_t As[kGT][kGK + 1];
    __shared__ uint32_t Bs[kGT][kGK + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    uint32_t acc[4][4] = {};
    for (int64_t kk = k0; kk < k1; kk += kGK) {
        for (int i = threadIdx.x; i < kGT * kGK; i += 256) {
            const int r = i / kGK, c = i % kGK;
            const int64_t k = kk + c;
            const int e = E * kGT + r, f = F * kGT + r;
            As[r][c] = (e < P && k < k1) ? Xt[(int64_t)e * nsp4 + k] : 0u;
            Bs[r][c] = (f < P && k < k1) ? Xt[(int64_t)f * nsp4 + k] : 0u;
        }
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < kGK; c++) {
            uint32_t a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                a[u] = As[ty * 4 + u][c];
                b[u] = Bs[tx * 4 + u][c];
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[u][v] = __builtin_amdgcn_udot4(a[u], b[v], acc[u][v], false);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int e = E * kGT + ty * 4 + u, f = F * kGT + tx * 4 + v;
            if (e < P && f < P && acc[u][v])
                atomicAdd((unsigned long long*)&gram[(int64_t)e * P + f],
                          (unsigned long long)acc[u][v]);
        }
}

// A_s[i][j] = n_sub * Sxx[e_i][e_j] - Sx[e_i] * Sx[e_j], exact in int64, then
// one correctly rounded conversion to double.
__global__ void cov_matrix_kernel(const uint64_t* __restrict__ sum,
                                  const uint64_t* __restrict__ gram, int64_t nsub, int P,
                                  const int32_t* __restrict__ elems, const int32_t* __restrict__ msz,
                                  int mmax, double* __restrict__ A) {
    const int s = blockIdx.y;
    const int m = msz[s];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)m * m) return;
    const int r = (int)(i / m), c = (int)(i % m);
    const int e = elems[s * mmax + r], f = elems[s * mmax + c];
    const int lo = min(e, f), hi = max(e, f);
    const int64_t a = nsub * (int64_t)gram[(int64_t)lo * P + hi] - (int64_t)sum[e] * (int64_t)sum[f];
    A[(int64_t)s * mmax * mmax + i] = (double)a;
}

// ------------------------------------------------------------ Jacobi
// One workgroup per subset. Rotations of one round act on disjoint index
// pairs (round-robin pairing), so each round is two data-parallel phases:
//   decide (c, s) per pair from the round's starting matrix;
//   A <- J^T A J (rows then columns, pair entries zeroed) and V <- V J.
// The operation sequence per element matches the documented algorithm
// exactly (no fused multiply-add: the file is compiled with contraction off).
constexpr int kJacThreads = 1024;
constexpr int kJacMaxPairs = (kMaxSubsetElems + 1) / 2 + 1;

__global__ __launch_bounds__(kJacThreads) void jacobi_kernel(double* __restrict__ Aall,
                                                              double* __restrict__ Vall,
                                                              double* __restrict__ Ball,
                                                              const int32_t* __restrict__ msz,
                                                              int mmax, int32_t* __restrict__ sweeps) {
    const int s = blockIdx.x;
    const int m = msz[s];
    double* A = Aall + (int64_t)s * mmax * mmax;
    double* V = Vall + (int64_t)s * mmax * mmax;
    double* B = Ball + (int64_t)s * mmax * mmax;
    const int M = m + (m & 1);
    const int np = M / 2;
    __shared__ int sp[kJacMaxPairs], sq[kJacMaxPairs], sact[kJacMaxPairs];
    __shared__ double scs[kJacMaxPairs], ssn[kJacMaxPairs];
    __shared__ double s_tiny;
    __shared__ int s_rot;
    const int tid = threadIdx.x;

    for (int64_t i = tid; i < (int64_t)m * m; i += kJacThreads) {
        const int r = (int)(i / m), c = (int)(i % m);
        V[i] = (r == c) ? 1.0 : 0.0;
    }
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < m; i++) {
            const double a = fabs(A[(int64_t)i * m + i]);
            if (a > t) t = a;
        }
        s_tiny = ldexp(t, -100);
    }
    __syncthreads();
    const double tiny = s_tiny;

    int sweep = 0;
    while (sweep < 60) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r = 0; r < M - 1; r++) {
            if (tid < np) {
                const int k = tid;
                int a, b;
                if (k == 0) {
                    a = r;
                    b = M - 1;
                } else {
                    a = (r + k) % (M - 1);
                    b = (r - k + (M - 1)) % (M - 1);
                }
                const int p = a < b ? a : b, q = a < b ? b : a;
                sp[k] = p;
                sq[k] = q;
                int act = 0;
                if (q < m) {
                    const double apq = A[(int64_t)p * m + q];
                    const double app = A[(int64_t)p * m + p], aqq = A[(int64_t)q * m + q];
                    const double g = 100.0 * fabs(apq);
                    if (fabs(apq) <= tiny || (fabs(app) + g == fabs(app) && fabs(aqq) + g == fabs(aqq))) {
                        A[(int64_t)p * m + q] = 0.0;
                        A[(int64_t)q * m + p] = 0.0;
                    } else {
                        const double theta = (aqq - app) / (2.0 * apq);
                        double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
                        if (theta < 0.0) t = -t;
                        const double c = 1.0 / sqrt(1.0 + t * t);
                        scs[k] = c;
                        ssn[k] = t * c;
                        act = 1;
                        atomicAdd(&s_rot, 1);
                    }
                }
                sact[k] = act;
            }
            __syncthreads();
            // A <- J^T A J block by block: the 2x2 block at (rows of pair k1,
            // columns of pair k2) depends only on itself. Rows are rotated
            // first (when pair k1 rotates), then columns (when pair k2
            // rotates), exactly the operations of the row pass followed by
            // the column pass; blocks are disjoint, so the update is in place.
            // V <- V J runs alongside on its own data.
            // blocks: item i = k1*np + k2 with i = tid + it*kJacThreads, the
            // pair indices advanced by constant steps (no division per item)
            {
                const int d1 = kJacThreads / np, d2 = kJacThreads % np;
                int k1 = tid / np, k2 = tid % np;
                constexpr int kBatch = 4;
                while (k1 < np) {
                    int bk1[kBatch], bk2[kBatch];
                    double x[kBatch][4];
#pragma unroll
                    for (int u = 0; u < kBatch; u++) {
                        bk1[u] = k1;
                        bk2[u] = k2;
                        if (k1 < np) {
                            const int r0 = sp[k1], r1 = sq[k1], c0 = sp[k2], c1 = sq[k2];
                            const bool vr1 = r1 < m, vc1 = c1 < m;
                            x[u][0] = A[r0 * m + c0];
                            x[u][1] = vc1 ? A[r0 * m + c1] : 0.0;
                            x[u][2] = vr1 ? A[r1 * m + c0] : 0.0;
                            x[u][3] = (vr1 && vc1) ? A[r1 * m + c1] : 0.0;
                        }
                        k1 += d1;
                        k2 += d2;
                        if (k2 >= np) {
                            k2 -= np;
                            k1++;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kBatch; u++) {
                        const int a1 = bk1[u], a2 = bk2[u];
                        if (a1 >= np) continue;
                        double x00 = x[u][0], x01 = x[u][1], x10 = x[u][2], x11 = x[u][3];
                        if (sact[a1]) {
                            const double c = scs[a1], sn = ssn[a1];
                            const double y00 = c * x00 - sn * x10, y10 = sn * x00 + c * x10;
                            const double y01 = c * x01 - sn * x11, y11 = sn * x01 + c * x11;
                            x00 = y00; x10 = y10; x01 = y01; x11 = y11;
                        }
                        if (sact[a2]) {
                            const double c = scs[a2], sn = ssn[a2];
                            const double y00 = c * x00 - sn * x01, y01 = sn * x00 + c * x01;
                            const double y10 = c * x10 - sn * x11, y11 = sn * x10 + c * x11;
                            x00 = y00; x01 = y01; x10 = y10; x11 = y11;
                        }
                        if (a1 == a2 && sact[a1]) {
                            x01 = 0.0;
                            x10 = 0.0;
                        }
                        const int r0 = sp[a1], r1 = sq[a1], c0 = sp[a2], c1 = sq[a2];
                        const bool vr1 = r1 < m, vc1 = c1 < m;
                        A[r0 * m + c0] = x00;
                        if (vc1) A[r0 * m + c1] = x01;
                        if (vr1) A[r1 * m + c0] = x10;
                        if (vr1 && vc1) A[r1 * m + c1] = x11;
                    }
                }
            }
            // eigenvectors: item i = k*m + j, same stepping, loads batched
            {
                const int d1 = kJacThreads / m, d2 = kJacThreads % m;
                int k = tid / m, j = tid % m;
                constexpr int kVB = 8;
                while (k < np) {
                    int bk[kVB], bj[kVB];
                    double xv[kVB], yv[kVB];
#pragma unroll
                    for (int u = 0; u < kVB; u++) {
                        bk[u] = k;
                        bj[u] = j;
                        if (k < np && sact[k]) {
                            xv[u] = V[j * m + sp[k]];
                            yv[u] = V[j * m + sq[k]];
                        }
                        k += d1;
                        j += d2;
                        if (j >= m) {
                            j -= m;
                            k++;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kVB; u++) {
                        const int kk = bk[u];
                        if (kk >= np || !sact[kk]) continue;
                        const double c = scs[kk], sn = ssn[kk];
                        V[bj[u] * m + sp[kk]] = c * xv[u] - sn * yv[u];
                        V[bj[u] * m + sq[kk]] = sn * xv[u] + c * yv[u];
                    }
                }
            }
            __syncthreads();
        }
        sweep++;
        const int rot = s_rot;
        __syncthreads();
        if (rot == 0) break;
    }
    if (tid == 0) sweeps[s] = sweep;
}

// First D components by eigenvalue (descending, ties to the lower column),
// largest-magnitude entry made positive, one scale g = max |v| per subset,
// w = rint(v * 127 / g).
__global__ __launch_bounds__(256) void basis_kernel(const double* __restrict__ Aall,
                                                    const double* __restrict__ Vall,
                                                    const int32_t* __restrict__ msz, int mmax,
                                                    int D, int8_t* __restrict__ basis) {
    const int s = blockIdx.x;
    const int m = msz[s];
    const double* A = Aall + (int64_t)s * mmax * mmax;
    const double* V = Vall + (int64_t)s * mmax * mmax;
    __shared__ int order[kMaxD];
    __shared__ double sgn[kMaxD];
    __shared__ double gmax;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double li = A[(int64_t)i * m + i];
        int rank = 0;
        for (int j = 0; j < m; j++) {
            const double lj = A[(int64_t)j * m + j];
            if (lj > li || (lj == li && j < i)) rank++;
        }
        if (rank < D) order[rank] = i;
    }
    __syncthreads();
    if ((int)threadIdx.x < D) {
        const int col = order[threadIdx.x];
        int best = 0;
        for (int i = 1; i < m; i++)
            if (fabs(V[(int64_t)i * m + col]) > fabs(V[(int64_t)best * m + col])) best = i;
        sgn[threadIdx.x] = (V[(int64_t)best * m + col] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double g = 0.0;
        for (int d = 0; d < D; d++)
            for (int i = 0; i < m; i++) {
                const double v = fabs(sgn[d] * V[(int64_t)i * m + order[d]]);
                if (v > g) g = v;
            }
        gmax = g;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m * D; i += blockDim.x) {
        const int r = i / D, d = i % D;
        const double v = sgn[d] * V[(int64_t)r * m + order[d]];
        basis[(int64_t)s * mmax * D + i] = (int8_t)rint((v * 127.0) / gmax);
    }
}

}  // namespace

sfc_status launch_quantize(const float* vol, const uint8_t* mask, const Grid& g, uint8_t* xq,
                           float* params, uint32_t* mm, hipStream_t st) {
    minmax_init_kernel<<<1, 1, 0, st>>>(mm);
    SFC_TRY(launched("minmax_init_kernel"));
    const unsigned nb = (unsigned)std::min<int64_t>(4096, (g.nvox + 255) / 256);
    minmax_kernel<<<nb, 256, 0, st>>>(vol, mask, g.nvox, g.C, mm);
    SFC_TRY(launched("minmax_kernel"));
    scale_kernel<<<1, 1, 0, st>>>(mm, params);
    SFC_TRY(launched("scale_kernel"));
    const int64_t n = g.nvox * g.C;
    quantize_kernel<<<blocks_for(n), 256, 0, st>>>(vol, n, params, xq);
    return launched("quantize_kernel");
}

sfc_status launch_gather_samples(const uint8_t* xq, const uint32_t* dict, int64_t stride,
                                 int64_t nsub, const int32_t* elem_off, int P, int C,
                                 uint32_t* Xt, int64_t nsp4, hipStream_t st) {
    gather_samples_kernel<<<blocks_for((int64_t)P * nsp4), 256, 0, st>>>(xq, dict, stride, nsub,
                                                                         elem_off, P, C, Xt, nsp4);
    return launched("gather_samples_kernel");
}

sfc_status launch_gram(const uint32_t* Xt, int P, int64_t nsp4, uint64_t* sum, uint64_t* gram,
                       hipStream_t st) {
    sample_sum_kernel<<<P, 256, 0, st>>>(Xt, nsp4, sum);
    SFC_TRY(launched("sample_sum_kernel"));
    const int nt = (P + kGT - 1) / kGT;
    const int pairs = nt * (nt + 1) / 2;
    const int64_t chunks = (nsp4 + kGChunk - 1) / kGChunk;
    if (chunks > 65535) return fail(SFC_EUNSUPPORTED, "gram: too many samples");
    gram_kernel<<<dim3(pairs, (unsigned)chunks), 256, 0, st>>>(Xt, P, nsp4, nt, gram);
    return launched("gram_kernel");
}

sfc_status launch_cov_matrix(const uint64_t* sum, const uint64_t* gram, int64_t nsub, int P,
                             const int32_t* elems, const int32_t* m, int S, int mmax, double* A,
                             hipStream_t st) {
    cov_matrix_kernel<<<dim3(blocks_for((int64_t)mmax * mmax), S), 256, 0, st>>>(
        sum, gram, nsub, P, elems, m, mmax, A);
    return launched("cov_matrix_kernel");
}

sfc_status launch_jacobi(double* A, double* V, double* B, const int32_t* m, int S, int mmax,
                         int32_t* sweeps, hipStream_t st) {
    if (mmax > kMaxSubsetElems) return fail(SFC_EUNSUPPORTED, "subset larger than 518 elements");
    jacobi_kernel<<<S, kJacThreads, 0, st>>>(A, V, B, m, mmax, sweeps);
    return launched("jacobi_kernel");
}

sfc_status launch_basis(const double* A, const double* V, const int32_t* m, int S, int mmax,
                        int D, int8_t* basis, hipStream_t st) {
    if (D > kMaxD) return fail(SFC_EUNSUPPORTED, "reduced dimension above 32");
    basis_kernel<<<S, 256, 0, st>>>(A, V, m, mmax, D, basis);
    return launched("basis_kernel");
}

}  // namespace sfc
