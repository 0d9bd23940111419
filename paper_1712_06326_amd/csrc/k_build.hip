// Index build, part 1 (Sections II, II.A): byte quantisation of the volume,
// exact integer patch statistics over a strided subsample of the dictionary,
// per-subset covariance, float64 Jacobi eigendecomposition and the int8
// basis of the first D principal components.
#include <mutex>

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

// min / max of the ordered encodings over a 256-thread block (results in
// thread 0)
__device__ inline void block_minmax(uint32_t& lo, uint32_t& hi) {
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
    }
    __shared__ uint32_t wl[4], wh[4];
    if ((threadIdx.x & 63) == 0) {
        wl[threadIdx.x >> 6] = lo;
        wh[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < 4; w++) {
            lo = min(lo, wl[w]);
            hi = max(hi, wh[w]);
        }
}

// per-block partial range of the known voxels: part[2b] = min, part[2b+1] =
// max of the ordered encodings (identity values for a block with none)
__global__ __launch_bounds__(256) void minmax_kernel(const float* __restrict__ vol,
                                                     const uint8_t* __restrict__ mask,
                                                     int64_t nvox, int C,
                                                     uint32_t* __restrict__ part) {
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
    block_minmax(lo, hi);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lo;
        part[2 * blockIdx.x + 1] = hi;
    }
}

// params = {vmin, scale = 255 / (vmax - vmin) in float32 (0 when the range is
// empty), vmax}, from the nb partial ranges (one 256-thread block)
__global__ __launch_bounds__(256) void scale_kernel(const uint32_t* __restrict__ part, int nb,
                                                    float* __restrict__ params) {
    uint32_t lo = 0xffffffffu, hi = 0u;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        lo = min(lo, part[2 * b]);
        hi = max(hi, part[2 * b + 1]);
    }
    block_minmax(lo, hi);
    if (threadIdx.x == 0) {
        const float vlo = fdec(lo), vhi = fdec(hi);
        params[0] = vlo;
        params[1] = (vhi > vlo) ? 255.0f / (vhi - vlo) : 0.0f;
        params[2] = vhi;
    }
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

// Order-free checksum of the byte codes of the known voxels: the sum, mod
// 2^64, of (code + 1) times a mixed hash of the element's position.
__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

__global__ __launch_bounds__(256) void code_checksum_kernel(const uint8_t* __restrict__ xq,
                                                            const uint8_t* __restrict__ mask,
                                                            int64_t nvox, int C,
                                                            unsigned long long* __restrict__ out) {
    unsigned long long acc = 0ull;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (!mask[v]) continue;
        for (int ch = 0; ch < C; ch++) {
            unsigned long long z = (unsigned long long)(v * C + ch) + 0x9e3779b97f4a7c15ull;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            z ^= z >> 31;
            acc += z * (unsigned long long)(xq[v * C + ch] + 1u);
        }
    }
    __shared__ unsigned long long part[256];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, part[0]);
}

// ------------------------------------------------------------ covariance
// Xt[e][s4] packs the bytes of samples 4*s4 .. 4*s4+3 of element e.
// One thread per (4-sample group s4, block of kSampleEls elements): the four
// centres are read once and serve every element of the block.
constexpr int kSampleEls = 8;
__global__ void gather_samples_kernel(const uint8_t* __restrict__ xq,
                                      const uint32_t* __restrict__ dict, int64_t stride,
                                      int64_t nsub, const int32_t* __restrict__ elem_off, int P,
                                      int C, uint32_t* __restrict__ Xt, int64_t nsp4) {
    const int64_t s4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s4 >= nsp4) return;
    int64_t base[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int64_t s = s4 * 4 + k;
        base[k] = s < nsub ? (int64_t)dict[s * stride] * C : -1;
    }
    const int e0 = (int)blockIdx.y * kSampleEls;
#pragma unroll
    for (int j = 0; j < kSampleEls; j++) {
        const int e = e0 + j;
        if (e >= P) break;
        const int64_t off = elem_off[e];
        uint32_t w = 0;
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (base[k] >= 0) w |= (uint32_t)xq[base[k] + off] << (8 * k);
        Xt[(int64_t)e * nsp4 + s4] = w;
    }
}

// sum[e] += the sample bytes of element e in chunk blockIdx.y of kSumChunk
// dwords (sum pre-zeroed; integer adds, so the order does not matter)
constexpr int kSumChunk = 4096;
__global__ __launch_bounds__(256) void sample_sum_kernel(const uint32_t* __restrict__ Xt,
                                                         int64_t nsp4,
                                                         unsigned long long* __restrict__ sum) {
    const int e = blockIdx.x;
    const int64_t k0 = (int64_t)blockIdx.y * kSumChunk;
    const int64_t k1 = k0 + kSumChunk < nsp4 ? k0 + kSumChunk : nsp4;
    uint32_t acc = 0;   // at most 16 dwords of 4 bytes per thread
    for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
        const uint32_t w = Xt[(int64_t)e * nsp4 + k];
        acc += (w & 0xff) + ((w >> 8) & 0xff) + ((w >> 16) & 0xff) + (w >> 24);
    }
    __shared__ uint32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&sum[e], (unsigned long long)red[0]);
}

constexpr int kGT = 64;        // gram tile (elements)
constexpr int kGChunk = 1024;  // dwords (4096 samples) per block: int32 partials cannot overflow

typedef int gram_i32x4 __attribute__((ext_vector_type(4)));
typedef int gram_i32x16 __attribute__((ext_vector_type(16)));
// 16-byte loads at dword alignment (global loads of this width need only
// dword alignment)
typedef gram_i32x4 gram_i32x4u __attribute__((aligned(4)));

// Centred Gram sums on the matrix cores: gram[e][f] += sum over the chunk of
// x'_e x'_f with x' = x - 128 as int8 (a byte XOR 0x80), for the 64 x 64
// tile pairs E <= F; each wave takes a 32 x 32 quarter of the pair on
// v_mfma_i32_32x32x32_i8. A chunk's int32 sums stay below 2^28 (16384
// samples of at most 2^14). Dwords past the chunk end enter as x' = 0; the
// zero bytes that pad the last dword are samples x = 0 and are counted by
// gram_offset_kernel, which adds 128 (S_e + S_f) - 2^14 N afterwards.
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
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = E * kGT + (wave >> 1) * 32 + (lane & 31);
    const int f = F * kGT + (wave & 1) * 32 + (lane & 31);
    const int kh = (lane >> 5) * 4;   // this half-wave's 4 dwords of a step
    const uint32_t* ra = Xt + (int64_t)min(e, P - 1) * nsp4;
    const uint32_t* rb = Xt + (int64_t)min(f, P - 1) * nsp4;
    gram_i32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; i++) acc[i] = 0;
    const gram_i32x4 centre = {(int)0x80808080u, (int)0x80808080u, (int)0x80808080u,
                               (int)0x80808080u};
    // whole steps (unrolled so that loads of later steps are in flight),
    // then the ragged last step with guarded loads
    const int64_t kfull = k0 + (k1 - k0) / 8 * 8;
    int64_t kd = k0;
#pragma unroll 4
    for (; kd < kfull; kd += 8) {
        const gram_i32x4 A = *reinterpret_cast<const gram_i32x4u*>(ra + kd + kh);
        const gram_i32x4 B = *reinterpret_cast<const gram_i32x4u*>(rb + kd + kh);
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A ^ centre, B ^ centre, acc, 0, 0, 0);
    }
    if (kd < k1) {
        const int64_t k = kd + kh;
        gram_i32x4 A, B;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            A[j] = k + j < k1 ? (int)ra[k + j] : (int)0x80808080u;
            B[j] = k + j < k1 ? (int)rb[k + j] : (int)0x80808080u;
        }
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A ^ centre, B ^ centre, acc, 0, 0, 0);
    }
    // lane holds column (lane & 31) of the quarter, rows (i/4)*8 + (lane/32)*4 + i%4
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int r = E * kGT + (wave >> 1) * 32 + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
        if (r < P && f < P && acc[i])
            atomicAdd((unsigned long long*)&gram[(int64_t)r * P + f],
                      (unsigned long long)(long long)acc[i]);
    }
}

// gram[e][f] (e <= f) from the centred sums: + 128 (S_e + S_f) - 2^14 N,
// N = the sample slots of every dword (the padding zeros included)
__global__ void gram_offset_kernel(uint64_t* __restrict__ gram, const uint64_t* __restrict__ sum,
                                   int P, int64_t nslots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)P * P) return;
    const int e = (int)(i / P), f = (int)(i % P);
    if (e > f) return;
    gram[i] += 128ull * (sum[e] + sum[f]) - 16384ull * (uint64_t)nslots;
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
// Round-robin Jacobi (disjoint pairs per round) on the packed upper triangle
// of each subset's symmetric matrix. Per round:
//   decide (c, s) per pair from the round's starting matrix, log it;
//   rotate every 2x2 block (rows of pair a, columns of pair b), a <= b, in
//   place: entry (x, y) above the diagonal is the row rotation of x's pair
//   followed by the column rotation of y's pair, the value the full-matrix
//   two-pass update gives above the diagonal (and mirrors below it).
// The triangle lives in LDS; when it is larger, its first rows stay in global
// memory. Eigenvectors are rebuilt afterwards by replaying the logged
// rotations on the rows of V, which are independent of each other.
// Arithmetic per entry matches the documented algorithm operation for
// operation (the file is compiled with contraction off).
constexpr int kJacThreads = 1024;
constexpr int kJacMaxPairs = (kMaxSubsetElems + 1) / 2 + 1;
constexpr int kJacTriLds = 19350;    // doubles of the triangle kept in LDS
constexpr int kJacChunk = 4;         // sweeps per launch (rotation-log depth)
constexpr int kJacMaxSweeps = 60;

// state per subset: [0] sweeps done, [1] converged, [2] sweeps in this chunk
struct JacState {
    int32_t done, conv, pad0, pad1;
    double tiny;
};

__device__ inline int tri_index(int x, int y, int m) {   // x <= y
    return x * (2 * m - x + 1) / 2 + (y - x);
}

// Entries [G, total) of the triangle in LDS, [0, G) in global memory
// (kSplit = false: G = 0, everything in LDS).
template <bool kSplit>
struct TriStore {
    double* lds;
    double* glob;
    int G, m;
    __device__ double get(int x, int y) const {
        const int t = x <= y ? tri_index(x, y, m) : tri_index(y, x, m);
        if (!kSplit) return lds[t];
        if (t >= G) return lds[t - G];
        return glob[t];
    }
    __device__ void set(int x, int y, double v) const {
        const int t = x <= y ? tri_index(x, y, m) : tri_index(y, x, m);
        if (!kSplit) lds[t] = v;
        else if (t >= G) lds[t - G] = v;
        else glob[t] = v;
    }
    // by packed position
    __device__ double at(int t) const {
        if (!kSplit) return lds[t];
        return t >= G ? lds[t - G] : glob[t];
    }
    __device__ void put(int t, double v) const {
        if (!kSplit) lds[t] = v;
        else if (t >= G) lds[t - G] = v;
        else glob[t] = v;
    }
};

// Pair of a round as the block phase needs it: indices and the offsets of
// their rows in the packed triangle (entry (x, y), x <= y, is at ro(x) + y).
struct JacPair {
    int p, q, rp, rq;
};

__device__ inline int tri_row_offset(int x, int m) { return x * (2 * m - x + 1) / 2 - x; }

// Off-diagonal block (rows of pair a, columns of pair b, a < b): the entry
// (x, y) above the diagonal takes the row rotation of x's pair, then the
// column rotation of y's pair. Inactive pairs (c < 0) rotate nothing.
template <bool kSplit>
__device__ inline void rotate_cross(const TriStore<kSplit>& T, const JacPair& A, const JacPair& B,
                                    double ca, double sa, double cb, double sb, int m) {
    const bool acta = ca >= 0.0, actb = cb >= 0.0;
    const bool va = A.q < m, vb = B.q < m;
    // packed positions of (pa,pb), (pa,qb), (qa,pb), (qa,qb)
    const int t00 = A.p < B.p ? A.rp + B.p : B.rp + A.p;
    const int t01 = A.p < B.q ? A.rp + B.q : B.rq + A.p;
    const int t10 = A.q < B.p ? A.rq + B.p : B.rp + A.q;
    const int t11 = A.q < B.q ? A.rq + B.q : B.rq + A.q;
    const double x00 = T.at(t00);
    const double x01 = vb ? T.at(t01) : 0.0;
    const double x10 = va ? T.at(t10) : 0.0;
    const double x11 = (va && vb) ? T.at(t11) : 0.0;
    // rows by a, then columns by b: Z
    double z00 = x00, z01 = x01, z10 = x10, z11 = x11;
    if (acta) {
        const double y00 = ca * z00 - sa * z10, y10 = sa * z00 + ca * z10;
        const double y01 = ca * z01 - sa * z11, y11 = sa * z01 + ca * z11;
        z00 = y00; z10 = y10; z01 = y01; z11 = y11;
    }
    if (actb) {
        const double y00 = cb * z00 - sb * z01, y01 = sb * z00 + cb * z01;
        const double y10 = cb * z10 - sb * z11, y11 = sb * z10 + cb * z11;
        z00 = y00; z01 = y01; z10 = y10; z11 = y11;
    }
    // rows by b, then columns by a, on the transposed block: W,
    // W[j][i] = new A(row j of pair b, column i of pair a)
    double w00 = x00, w01 = x10, w10 = x01, w11 = x11;
    if (actb) {
        const double y00 = cb * w00 - sb * w10, y10 = sb * w00 + cb * w10;
        const double y01 = cb * w01 - sb * w11, y11 = sb * w01 + cb * w11;
        w00 = y00; w10 = y10; w01 = y01; w11 = y11;
    }
    if (acta) {
        const double y00 = ca * w00 - sa * w01, y01 = sa * w00 + ca * w01;
        const double y10 = ca * w10 - sa * w11, y11 = sa * w10 + ca * w11;
        w00 = y00; w01 = y01; w10 = y10; w11 = y11;
    }
    T.put(t00, A.p < B.p ? z00 : w00);
    if (vb) T.put(t01, A.p < B.q ? z01 : w10);
    if (va) T.put(t10, A.q < B.p ? z10 : w01);
    if (va && vb) T.put(t11, A.q < B.q ? z11 : w11);
}

// pair k of round r (M even): (r, M-1) for k = 0, else ((r+k), (r-k)) mod M-1
__device__ inline void round_pair(int r, int k, int M, int* p, int* q) {
    int a, b;
    if (k == 0) {
        a = r;
        b = M - 1;
    } else {
        a = r + k;
        if (a >= M - 1) a -= M - 1;
        b = r - k;
        if (b < 0) b += M - 1;
    }
    *p = a < b ? a : b;
    *q = a < b ? b : a;
}

__global__ __launch_bounds__(256) void jacobi_init_kernel(const double* __restrict__ Aall,
                                                          double* __restrict__ Vall,
                                                          double* __restrict__ Tall,
                                                          const int32_t* __restrict__ msz, int mmax,
                                                          int64_t tri_stride,
                                                          JacState* __restrict__ state) {
    const int s = blockIdx.y;
    const int m = msz[s];
    const double* A = Aall + (int64_t)s * mmax * mmax;
    double* V = Vall + (int64_t)s * mmax * mmax;
    double* T = Tall + (int64_t)s * tri_stride;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)m * m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / m), c = (int)(i % m);
        V[i] = (r == c) ? 1.0 : 0.0;
        if (r <= c) T[tri_index(r, c, m)] = A[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < m; i++) {
            const double a = fabs(A[(int64_t)i * m + i]);
            if (a > t) t = a;
        }
        state[s] = JacState{0, 0, 0, 0, ldexp(t, -100)};
    }
}

template <bool kSplit>
__global__ __launch_bounds__(kJacThreads) void jacobi_sweeps_kernel(
    double* __restrict__ Tall, int64_t tri_stride, const int32_t* __restrict__ msz,
    JacState* __restrict__ state, double2* __restrict__ logall, int64_t log_stride,
    int32_t* __restrict__ nsw_out) {
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    if (state[s].conv) {
        if (tid == 0) nsw_out[s] = 0;
        return;
    }
    const int m = msz[s];
    const int M = m + (m & 1);
    const int np = M / 2;
    const int total = m * (m + 1) / 2;
    const int G = total > kJacTriLds ? total - kJacTriLds : 0;
    __shared__ double lds[kJacTriLds];
    __shared__ JacPair spair[kJacMaxPairs];
    __shared__ double2 scs[kJacMaxPairs];   // (c, s); c < 0: no rotation
    __shared__ int s_rot;
    double* Tg = Tall + (int64_t)s * tri_stride;
    double2* log = logall + (int64_t)s * log_stride;
    for (int t = G + tid; t < total; t += kJacThreads) lds[t - G] = Tg[t];
    const TriStore<kSplit> T{lds, Tg, G, m};
    const double tiny = state[s].tiny;
    const int done0 = state[s].done;
    // this thread's blocks: items u = tid + k * kJacThreads of the block
    // enumeration, (r, c) = (u / np, u % np) stepped without division
    const int nblk = np * (np - 1) / 2;
    const int nfull = (np & 1) ? nblk : np * (np / 2 - 1);
    const int dr = kJacThreads / np, dc = kJacThreads % np;
    const int r0 = tid / np, c0 = tid % np;
    __syncthreads();

    int sw = 0;
    bool conv = false;
    while (sw < kJacChunk && done0 + sw < kJacMaxSweeps) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r = 0; r < M - 1; r++) {
            if (tid < np) {
                // decide this pair's rotation and apply it to the pair's own
                // 2x2 diagonal block (both passes; a_pq -> 0)
                const int k = tid;
                int p, q;
                round_pair(r, k, M, &p, &q);
                double c = -1.0, sn = 0.0;
                if (q < m) {
                    const double apq = T.get(p, q);
                    const double app = T.get(p, p), aqq = T.get(q, q);
                    const double g = 100.0 * fabs(apq);
                    if (fabs(apq) <= tiny || (fabs(app) + g == fabs(app) && fabs(aqq) + g == fabs(aqq))) {
                        T.set(p, q, 0.0);
                    } else {
                        const double theta = (aqq - app) / (2.0 * apq);
                        double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
                        if (theta < 0.0) t = -t;
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                        const double y00 = c * app - sn * apq, y01 = c * apq - sn * aqq;
                        const double y10 = sn * app + c * apq, y11 = sn * apq + c * aqq;
                        T.set(p, p, c * y00 - sn * y01);
                        T.set(q, q, sn * y10 + c * y11);
                        T.set(p, q, 0.0);
                        atomicAdd(&s_rot, 1);
                    }
                }
                spair[k] = JacPair{p, q, tri_row_offset(p, m), q < m ? tri_row_offset(q, m) : 0};
                scs[k] = make_double2(c, sn);
                log[((int64_t)sw * (M - 1) + r) * np + k] = make_double2(c, sn);
            }
            __syncthreads();
            {
                // the np (np - 1) / 2 blocks a < b, by cyclic distance: row r
                // of an np-wide rectangle pairs c with (c + r + 1) mod np;
                // for even np a last half row holds the pairs np / 2 apart
                int r = r0, c = c0;
                for (int u = tid; u < nblk; u += kJacThreads) {
                    int a, b;
                    if (u < nfull) {
                        int y = c + r + 1;
                        if (y >= np) y -= np;
                        a = c < y ? c : y;
                        b = c < y ? y : c;
                    } else {
                        a = u - nfull;
                        b = a + np / 2;
                    }
                    const double2 ea = scs[a], eb = scs[b];
                    if (ea.x >= 0.0 || eb.x >= 0.0)
                        rotate_cross(T, spair[a], spair[b], ea.x, ea.y, eb.x, eb.y, m);
                    r += dr;
                    c += dc;
                    if (c >= np) {
                        c -= np;
                        r++;
                    }
                }
            }
            __syncthreads();
        }
        sw++;
        if (s_rot == 0) {
            conv = true;
            break;
        }
        __syncthreads();
    }
    __syncthreads();
    for (int t = G + tid; t < total; t += kJacThreads) Tg[t] = lds[t - G];
    if (tid == 0) {
        state[s].done = done0 + sw;
        nsw_out[s] = sw;
        state[s].conv = (conv || done0 + sw >= kJacMaxSweeps) ? 1 : 0;
    }
}

// V <- V J for the logged rounds: one wave per row of V, the row in LDS; the
// workgroup stages a batch of rounds' (c, s) in LDS for all its rows.
constexpr int kRepRows = 16;
constexpr int kRepStage = 4096;   // (c, s) entries staged per batch

__global__ __launch_bounds__(kRepRows * 64) void jacobi_replay_kernel(
    double* __restrict__ Vall, const int32_t* __restrict__ msz, int mmax,
    const int32_t* __restrict__ nsw_in, const double2* __restrict__ logall, int64_t log_stride) {
    const int s = blockIdx.y;
    const int nsw = nsw_in[s];
    const int m = msz[s];
    const int row0 = blockIdx.x * kRepRows;
    if (nsw == 0 || row0 >= m) return;
    const int M = m + (m & 1);
    const int np = M / 2;
    __shared__ double rows[kRepRows][kMaxSubsetElems];
    __shared__ double2 stage[kRepStage];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = row0 + wave;
    double* V = Vall + (int64_t)s * mmax * mmax;
    const double2* log = logall + (int64_t)s * log_stride;
    if (row < m)
        for (int j = lane; j < m; j += 64) rows[wave][j] = V[(int64_t)row * m + j];
    const int rounds = nsw * (M - 1);
    const int per = kRepStage / np;   // rounds per batch (np <= 260)
    for (int base = 0; base < rounds; base += per) {
        const int nr = min(per, rounds - base);
        __syncthreads();
        for (int i = threadIdx.x; i < nr * np; i += blockDim.x)
            stage[i] = log[(int64_t)base * np + i];
        __syncthreads();
        if (row < m) {
            for (int rr = 0; rr < nr; rr++) {
                const int r = (base + rr) % (M - 1);
                for (int k = lane; k < np; k += 64) {
                    const double2 cs = stage[rr * np + k];
                    if (cs.x < 0.0) continue;
                    int p, q;
                    round_pair(r, k, M, &p, &q);
                    const double x = rows[wave][p], y = rows[wave][q];
                    rows[wave][p] = cs.x * x - cs.y * y;
                    rows[wave][q] = cs.y * x + cs.x * y;
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    if (row < m)
        for (int j = lane; j < m; j += 64) V[(int64_t)row * m + j] = rows[wave][j];
}

__global__ void jacobi_finish_kernel(double* __restrict__ Aall, const double* __restrict__ Tall,
                                     int64_t tri_stride, const int32_t* __restrict__ msz, int mmax,
                                     const JacState* __restrict__ state,
                                     int32_t* __restrict__ sweeps) {
    const int s = blockIdx.x;
    const int m = msz[s];
    double* A = Aall + (int64_t)s * mmax * mmax;
    const double* T = Tall + (int64_t)s * tri_stride;
    for (int i = threadIdx.x; i < m; i += blockDim.x) A[(int64_t)i * m + i] = T[tri_index(i, i, m)];
    if (threadIdx.x == 0) sweeps[s] = state[s].done;
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
    const unsigned nb =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>(kQuantBlocks, (g.nvox + 255) / 256));
    minmax_kernel<<<nb, 256, 0, st>>>(vol, mask, g.nvox, g.C, mm);
    SFC_TRY(launched("minmax_kernel"));
    scale_kernel<<<1, 256, 0, st>>>(mm, (int)nb, params);
    SFC_TRY(launched("scale_kernel"));
    const int64_t n = g.nvox * g.C;
    quantize_kernel<<<blocks_for(n), 256, 0, st>>>(vol, n, params, xq);
    return launched("quantize_kernel");
}

sfc_status launch_code_checksum(const uint8_t* xq, const uint8_t* mask, int64_t nvox, int C,
                                uint64_t* out, hipStream_t st) {
    auto* o = reinterpret_cast<unsigned long long*>(out);
    zero_u64_kernel<<<1, 1, 0, st>>>(o);
    SFC_TRY(launched("zero_u64_kernel"));
    const unsigned nb = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (nvox + 255) / 256));
    code_checksum_kernel<<<nb, 256, 0, st>>>(xq, mask, nvox, C, o);
    return launched("code_checksum_kernel");
}

sfc_status launch_gather_samples(const uint8_t* xq, const uint32_t* dict, int64_t stride,
                                 int64_t nsub, const int32_t* elem_off, int P, int C,
                                 uint32_t* Xt, int64_t nsp4, hipStream_t st) {
    const unsigned eblocks = (unsigned)((P + kSampleEls - 1) / kSampleEls);
    gather_samples_kernel<<<dim3(blocks_for(nsp4), eblocks), 256, 0, st>>>(xq, dict, stride, nsub,
                                                                           elem_off, P, C, Xt,
                                                                           nsp4);
    return launched("gather_samples_kernel");
}

sfc_status launch_gram(const uint32_t* Xt, int P, int64_t nsp4, uint64_t* sum, uint64_t* gram,
                       hipStream_t st) {
    const int nt = (P + kGT - 1) / kGT;
    const int pairs = nt * (nt + 1) / 2;
    const int64_t chunks = (nsp4 + kGChunk - 1) / kGChunk;
    if (chunks > 65535) return fail(SFC_EUNSUPPORTED, "gram: too many samples");
    const int64_t schunks = (nsp4 + kSumChunk - 1) / kSumChunk;
    sample_sum_kernel<<<dim3(P, (unsigned)std::max<int64_t>(1, schunks)), 256, 0, st>>>(
        Xt, nsp4, reinterpret_cast<unsigned long long*>(sum));
    SFC_TRY(launched("sample_sum_kernel"));
    gram_kernel<<<dim3(pairs, (unsigned)chunks), 256, 0, st>>>(Xt, P, nsp4, nt, gram);
    SFC_TRY(launched("gram_kernel"));
    gram_offset_kernel<<<blocks_for((int64_t)P * P), 256, 0, st>>>(gram, sum, P, 4 * nsp4);
    return launched("gram_offset_kernel");
}

sfc_status launch_cov_matrix(const uint64_t* sum, const uint64_t* gram, int64_t nsub, int P,
                             const int32_t* elems, const int32_t* m, int S, int mmax, double* A,
                             hipStream_t st) {
    cov_matrix_kernel<<<dim3(blocks_for((int64_t)mmax * mmax), S), 256, 0, st>>>(
        sum, gram, nsub, P, elems, m, mmax, A);
    return launched("cov_matrix_kernel");
}

namespace {
// Two rotation logs and two per-launch sweep-count arrays: the replay of
// launch c reads buffer c % 2 while launch c + 1 writes the other one.
struct JacScratch {
    size_t tri, log, state, nsw;
};
JacScratch jacobi_layout(int S, int mmax) {
    const int64_t Mx = mmax + (mmax & 1);
    auto r256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    JacScratch L;
    L.tri = r256((size_t)S * ((size_t)mmax * (mmax + 1) / 2) * sizeof(double));
    L.log = r256((size_t)S * kJacChunk * (Mx - 1) * (Mx / 2) * sizeof(double2));
    L.state = r256((size_t)S * sizeof(JacState));
    L.nsw = r256((size_t)S * sizeof(int32_t));
    return L;
}

// The replays run on a second stream of the library (one per device,
// default priority), so that replaying one launch's rotations overlaps the
// next launch's sweeps.
std::mutex g_aux_mu;
hipStream_t g_aux[64] = {};
sfc_status aux_stream(hipStream_t* out) {
    int dev = 0;
    SFC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(SFC_EUNSUPPORTED, "device ordinal above 63");
    if (!g_aux[dev]) SFC_HIP(hipStreamCreateWithFlags(&g_aux[dev], hipStreamNonBlocking));
    *out = g_aux[dev];
    return SFC_OK;
}
}  // namespace

size_t jacobi_scratch_bytes(int S, int mmax) {
    const JacScratch L = jacobi_layout(S, mmax);
    return L.tri + 2 * L.log + L.state + 2 * L.nsw;
}

sfc_status launch_jacobi(double* A, double* V, void* scratch, const int32_t* m, int S, int mmax,
                         int32_t* sweeps, hipStream_t st) {
    if (mmax > kMaxSubsetElems) return fail(SFC_EUNSUPPORTED, "subset larger than 518 elements");
    const int64_t Mx = mmax + (mmax & 1);
    const int64_t tri_stride = (int64_t)mmax * (mmax + 1) / 2;
    const int64_t log_stride = (int64_t)kJacChunk * (Mx - 1) * (Mx / 2);
    const JacScratch L = jacobi_layout(S, mmax);
    char* base = static_cast<char*>(scratch);
    double* T = reinterpret_cast<double*>(base);
    double2* lg[2] = {reinterpret_cast<double2*>(base + L.tri),
                      reinterpret_cast<double2*>(base + L.tri + L.log)};
    JacState* state = reinterpret_cast<JacState*>(base + L.tri + 2 * L.log);
    int32_t* nsw[2] = {reinterpret_cast<int32_t*>(base + L.tri + 2 * L.log + L.state),
                       reinterpret_cast<int32_t*>(base + L.tri + 2 * L.log + L.state + L.nsw)};
    jacobi_init_kernel<<<dim3(blocks_for((int64_t)mmax * mmax), S), 256, 0, st>>>(A, V, T, m, mmax,
                                                                                 tri_stride, state);
    SFC_TRY(launched("jacobi_init_kernel"));
    auto hs = [](hipError_t e, const char* what) { return e == hipSuccess ? SFC_OK : check_hip(e, what); };
    std::lock_guard<std::mutex> lock(g_aux_mu);
    hipStream_t aux = nullptr;
    SFC_TRY(aux_stream(&aux));
    // swept[b]: launch c (c % 2 == b) has written log b; replayed[b]: its
    // replay has read log b (launch c + 2 may overwrite it)
    hipEvent_t ev[5] = {};
    sfc_status status = SFC_OK;
    for (auto& e : ev) {
        const hipError_t he = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (he != hipSuccess) status = hs(he, "hipEventCreateWithFlags");
    }
    hipEvent_t* swept = ev;
    hipEvent_t* replayed = ev + 2;
    hipEvent_t ready = ev[4];
    // the replays may start once V is initialised
    if (status == SFC_OK) status = hs(hipEventRecord(ready, st), "hipEventRecord");
    if (status == SFC_OK) status = hs(hipStreamWaitEvent(aux, ready, 0), "hipStreamWaitEvent");
    const unsigned rblocks = (unsigned)((mmax + kRepRows - 1) / kRepRows);
    const int chunks = (kJacMaxSweeps + kJacChunk - 1) / kJacChunk;
    for (int c = 0; c < chunks && status == SFC_OK; c++) {
        const int b = c & 1;
        if (c >= 2) status = hs(hipStreamWaitEvent(st, replayed[b], 0), "hipStreamWaitEvent");
        if (status != SFC_OK) break;
        if (tri_stride > kJacTriLds)
            jacobi_sweeps_kernel<true><<<S, kJacThreads, 0, st>>>(T, tri_stride, m, state, lg[b],
                                                                  log_stride, nsw[b]);
        else
            jacobi_sweeps_kernel<false><<<S, kJacThreads, 0, st>>>(T, tri_stride, m, state, lg[b],
                                                                   log_stride, nsw[b]);
        status = launched("jacobi_sweeps_kernel");
        if (status == SFC_OK) status = hs(hipEventRecord(swept[b], st), "hipEventRecord");
        if (status == SFC_OK) status = hs(hipStreamWaitEvent(aux, swept[b], 0), "hipStreamWaitEvent");
        if (status != SFC_OK) break;
        jacobi_replay_kernel<<<dim3(rblocks, S), kRepRows * 64, 0, aux>>>(V, m, mmax, nsw[b], lg[b],
                                                                         log_stride);
        status = launched("jacobi_replay_kernel");
        if (status == SFC_OK) status = hs(hipEventRecord(replayed[b], aux), "hipEventRecord");
    }
    // the caller's stream continues once the last replay is done (with an
    // error above, after whatever was enqueued)
    const int last = (chunks - 1) & 1;
    if (status == SFC_OK) status = hs(hipStreamWaitEvent(st, replayed[last], 0), "hipStreamWaitEvent");
    else (void)hipStreamSynchronize(aux);
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    SFC_TRY(status);
    jacobi_finish_kernel<<<S, 256, 0, st>>>(A, T, tri_stride, m, mmax, state, sweeps);
    return launched("jacobi_finish_kernel");
}

sfc_status launch_basis(const double* A, const double* V, const int32_t* m, int S, int mmax,
                        int D, int8_t* basis, hipStream_t st) {
    if (D > kMaxD) return fail(SFC_EUNSUPPORTED, "reduced dimension above 32");
    basis_kernel<<<S, 256, 0, st>>>(A, V, m, mmax, D, basis);
    return launched("basis_kernel");
}

}  // namespace sfc
