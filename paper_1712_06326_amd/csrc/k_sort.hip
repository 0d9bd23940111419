// Stable LSD radix sort of (multi-word key, 32-bit id) pairs: the order of
// a curve's entries by curve position (Section II.C). Ids enter in ascending
// order, so the result is ordered by (key, id).
//
// One pass per 8-bit digit that varies over the input (digits shared by all
// keys cannot change the order and are skipped). Per pass: per-tile digit
// counts, a per-digit scan over tiles, a scan over digit totals, and a
// scatter in which each tile ranks its items stably with wave-level
// multi-split (8 ballots give each lane its peers with the same digit) and a
// per-round prefix over the four waves held in LDS.
#include <algorithm>
#include <utility>

#include "proj.hpp"

namespace sfc {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kTileItems = kThreads * kRounds;   // 4096

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

sfc_status launched(const char* what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, what);
}

__device__ inline uint32_t digit_of(const uint64_t* keys, int64_t n, int64_t i, int W64, int pb) {
    const int w = W64 - 1 - (pb >> 6);
    return (uint32_t)((keys[(int64_t)w * n + i] >> (pb & 63)) & 0xffu);
}

__global__ __launch_bounds__(kThreads) void hist_kernel(const uint64_t* __restrict__ keys_all, int64_t n,
                                                        int W64, int pb, int64_t nb,
                                                        uint32_t* __restrict__ counts_all) {
    const uint64_t* keys = keys_all + (int64_t)blockIdx.y * W64 * n;
    uint32_t* counts = counts_all + (int64_t)blockIdx.y * 256 * nb;
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTileItems;
    for (int k = 0; k < kRounds; k++) {
        const int64_t i = t0 + (int64_t)k * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[digit_of(keys, n, i, W64, pb)], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of counts[d][0..nb) in place (one block per digit);
// totals[d] = the digit's count.
__global__ __launch_bounds__(kThreads) void scan_digit_kernel(uint32_t* __restrict__ counts_all,
                                                              int64_t nb,
                                                              uint32_t* __restrict__ totals_all) {
    const int d = blockIdx.x;
    uint32_t* row = counts_all + (int64_t)blockIdx.y * 256 * nb + (int64_t)d * nb;
    uint32_t* totals = totals_all + blockIdx.y * 256;
    __shared__ uint32_t wsum[kThreads / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t x = i < nb ? row[i] : 0u;
        uint32_t inc = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        for (int k = 0; k < kThreads / 64; k++) {
            if (k < w) pre += wsum[k];
            tot += wsum[k];
        }
        const uint32_t c = carry;
        if (i < nb) row[i] = c + pre + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[d] = carry;
}

__global__ void digit_base_kernel(const uint32_t* __restrict__ totals_all,
                                  uint32_t* __restrict__ dbase_all) {
    const uint32_t* totals = totals_all + blockIdx.x * 256;
    uint32_t* dbase = dbase_all + blockIdx.x * 256;
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int d = 0; d < 256; d++) {
            dbase[d] = acc;
            acc += totals[d];
        }
    }
}

// Scatter of one tile: local stable ranks by wave multi-split, then each
// key word (and the ids) is reordered by digit in LDS and written out in
// digit runs, so global writes are contiguous within each run.
__global__ __launch_bounds__(kThreads) void scatter_kernel(
    const uint64_t* __restrict__ kin_all, const uint32_t* __restrict__ iin_all,
    uint64_t* __restrict__ kout_all, uint32_t* __restrict__ iout_all, int64_t n, int W64, int pb,
    int64_t nb, const uint32_t* __restrict__ counts_all, const uint32_t* __restrict__ dbase_all) {
    const int64_t arr = blockIdx.y;
    const uint64_t* kin = kin_all + arr * W64 * n;
    uint64_t* kout = kout_all + arr * W64 * n;
    const uint32_t* iin = iin_all + arr * n;
    uint32_t* iout = iout_all + arr * n;
    const uint32_t* counts = counts_all + arr * 256 * nb;
    const uint32_t* dbase = dbase_all + arr * 256;
    __shared__ uint32_t cnt[kThreads / 64][256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t tbase[256];
    __shared__ uint32_t wsum[kThreads / 64];
    __shared__ uint8_t sdig[kTileItems];
    __shared__ uint64_t sval[kTileItems];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kTileItems;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    uint32_t dg[kRounds];
    run[tid] = 0;
    tstart[tid] = 0;
    tbase[tid] = dbase[tid] + counts[(int64_t)tid * nb + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRounds; k++) {
        const int64_t i = t0 + (int64_t)k * kThreads + tid;
        dg[k] = (i < n) ? digit_of(kin, n, i, W64, pb) : 0xffffffffu;
        if (i < n) atomicAdd(&tstart[dg[k]], 1u);
    }
    __syncthreads();
    {
        // exclusive scan of the tile's digit counts (thread tid owns digit tid)
        const uint32_t x = tstart[tid];
        uint32_t inc = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
        for (int k = 0; k < w; k++) pre += wsum[k];
        tstart[tid] = pre + inc - x;
    }
    uint32_t lp[kRounds];
#pragma unroll
    for (int k = 0; k < kRounds; k++) {
        for (int ww = 0; ww < kThreads / 64; ww++) cnt[ww][tid] = 0;
        __syncthreads();
        const bool valid = dg[k] != 0xffffffffu;
        const uint32_t d = valid ? dg[k] : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bl = __ballot(on);
            peers &= on ? bl : ~bl;
        }
        const uint32_t rk = (uint32_t)__popcll(peers & lt);
        if (valid && rk == 0) cnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t acc = run[tid];
            for (int ww = 0; ww < kThreads / 64; ww++) {
                const uint32_t c = cnt[ww][tid];
                cnt[ww][tid] = acc;
                acc += c;
            }
            run[tid] = acc;
        }
        __syncthreads();
        lp[k] = valid ? tstart[d] + cnt[w][d] + rk : 0xffffffffu;
        if (valid) sdig[lp[k]] = (uint8_t)d;
        __syncthreads();   // cnt is cleared by the next round
    }
    __syncthreads();
    const int64_t tn = min((int64_t)kTileItems, n - t0);
    for (int x = 0; x <= W64; x++) {
#pragma unroll
        for (int k = 0; k < kRounds; k++) {
            if (lp[k] == 0xffffffffu) continue;
            const int64_t i = t0 + (int64_t)k * kThreads + tid;
            sval[lp[k]] = (x < W64) ? kin[(int64_t)x * n + i] : (uint64_t)iin[i];
        }
        __syncthreads();
        for (int slot = tid; slot < tn; slot += kThreads) {
            const uint32_t d = sdig[slot];
            const int64_t gpos = (int64_t)tbase[d] + slot - tstart[d];
            if (x < W64) kout[(int64_t)x * n + gpos] = sval[slot];
            else iout[gpos] = (uint32_t)sval[slot];
        }
        __syncthreads();
    }
}

__global__ void varying_kernel(const uint64_t* __restrict__ keys, int64_t n, int W64,
                               uint64_t* __restrict__ varying) {
    const int arr = blockIdx.y;
    const uint64_t* k = keys + (int64_t)arr * W64 * n;
    for (int w = 0; w < W64; w++) {
        const uint64_t k0 = k[(int64_t)w * n];
        uint64_t acc = 0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            acc |= k[(int64_t)w * n + i] ^ k0;
        for (int off = 32; off > 0; off >>= 1) acc |= (uint64_t)__shfl_xor((long long)acc, off, 64);
        if ((threadIdx.x & 63) == 0 && acc)
            atomicOr((unsigned long long*)&varying[arr * W64 + w], (unsigned long long)acc);
    }
}

}  // namespace

size_t sort_scratch_bytes(int64_t n, int W64, int arrays) {
    const int64_t nb = (n + kTileItems - 1) / kTileItems;
    return (size_t)arrays * ((size_t)n * (8 * W64 + 4) + (size_t)(256 * nb + 512) * 4) + 256;
}

sfc_status launch_varying_bits(const uint64_t* keys, int64_t n, int W64, int arrays,
                               uint64_t* varying, hipStream_t st) {
    if (n == 0 || arrays == 0) return SFC_OK;
    const unsigned nb = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
    varying_kernel<<<dim3(nb, arrays), 256, 0, st>>>(keys, n, W64, varying);
    return launched("varying_kernel");
}

sfc_status radix_sort(uint64_t* keys, uint32_t* ids, int64_t n, int W64, int arrays,
                      const SortPlan& plan, void* scratch, hipStream_t st) {
    if (n <= 1 || plan.n_passes == 0 || arrays == 0) return SFC_OK;
    const int64_t nb = (n + kTileItems - 1) / kTileItems;
    char* p = static_cast<char*>(scratch);
    uint64_t* k2 = reinterpret_cast<uint64_t*>(p);
    p += (size_t)arrays * n * 8 * W64;
    uint32_t* i2 = reinterpret_cast<uint32_t*>(p);
    p += (size_t)arrays * n * 4;
    p = reinterpret_cast<char*>(((uintptr_t)p + 255) & ~uintptr_t(255));
    uint32_t* counts = reinterpret_cast<uint32_t*>(p);
    uint32_t* totals = counts + (size_t)arrays * 256 * nb;
    uint32_t* dbase = totals + (size_t)arrays * 256;
    uint64_t *kin = keys, *kout = k2;
    uint32_t *iin = ids, *iout = i2;
    if (nb > 0x7fffffff || arrays > 65535) return fail(SFC_EUNSUPPORTED, "sort grid too large");
    for (int ps = 0; ps < plan.n_passes; ps++) {
        const int pb = plan.pass_bits[ps];
        hist_kernel<<<dim3((unsigned)nb, arrays), kThreads, 0, st>>>(kin, n, W64, pb, nb, counts);
        SFC_TRY(launched("hist_kernel"));
        scan_digit_kernel<<<dim3(256, arrays), kThreads, 0, st>>>(counts, nb, totals);
        SFC_TRY(launched("scan_digit_kernel"));
        digit_base_kernel<<<arrays, 64, 0, st>>>(totals, dbase);
        SFC_TRY(launched("digit_base_kernel"));
        scatter_kernel<<<dim3((unsigned)nb, arrays), kThreads, 0, st>>>(kin, iin, kout, iout, n, W64,
                                                                        pb, nb, counts, dbase);
        SFC_TRY(launched("scatter_kernel"));
        std::swap(kin, kout);
        std::swap(iin, iout);
    }
    if (kin != keys) {
        SFC_HIP(hipMemcpyAsync(keys, kin, (size_t)arrays * n * 8 * W64, hipMemcpyDeviceToDevice, st));
        SFC_HIP(hipMemcpyAsync(ids, iin, (size_t)arrays * n * 4, hipMemcpyDeviceToDevice, st));
    }
    return SFC_OK;
}

}  // namespace sfc
