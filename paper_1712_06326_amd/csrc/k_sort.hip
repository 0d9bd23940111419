// Stable LSD radix sort of (multi-word key, 32-bit id) pairs: the order of
// a curve's entries by curve position (Section II.C). Ids enter in ascending
// order, so the result is ordered by (key, id).
//
// One pass per 8-bit digit that varies over the input (digits shared by all
// keys cannot change the order and are skipped). Per pass: per-tile digit
// counts, a per-digit scan over tiles, a scan over digit totals, and a
// scatter in which each tile ranks its items stably with wave-level
// multi-split (8 ballots give each lane its peers with the same digit).
//
// Every pass carries one 64-bit key word and a 32-bit payload. When a single
// word varies, the payload is the id and that word is the only one moved.
// When several do, the passes of a word carry the word and the item's
// original position (its rank); the next word is gathered by rank before its
// passes, and after the last pass the ids and every varying word are
// gathered once by the final ranks. A pass over three words at once would
// move 28 bytes per item each way instead of 12.
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

// Digit counts per tile of 4096 items. Array a's digit word starts at
// keys_all + a * ks.
__global__ __launch_bounds__(kThreads) void hist_kernel(const uint64_t* __restrict__ keys_all,
                                                        int64_t ks, int64_t n, int sh, int64_t nb,
                                                        uint32_t* __restrict__ counts_all) {
    const uint64_t* keys = keys_all + (int64_t)blockIdx.y * ks;
    uint32_t* counts = counts_all + (int64_t)blockIdx.y * 256 * nb;
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTileItems;
    for (int k = 0; k < kRounds; k++) {
        const int64_t i = t0 + (int64_t)k * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> sh) & 0xffu], 1u);
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

// Scatter of one tile of (key word, payload) items; array a's words start at
// kin_all + a * ksi and kout_all + a * kso, its payloads at a * n (a null
// pin means payload = item index). Wave w ranks the tile's w-th quarter
// (items in order, 64 per round) against wave-private digit counters in LDS:
// the lowest peer with a digit adds the group's size to the counter and
// hands the old value to the others. No barrier is needed until the
// quarters are merged into per-(wave, digit) offsets, and since quarters are
// in item order the ranks are stable. The words and then the payloads are
// reordered by digit in LDS and written out in digit runs, so global writes
// are contiguous within each run.
__global__ __launch_bounds__(kThreads) void scatter_kernel(
    const uint64_t* __restrict__ kin_all, int64_t ksi, uint64_t* __restrict__ kout_all,
    int64_t kso, const uint32_t* __restrict__ pin_all, uint32_t* __restrict__ pout_all, int64_t n,
    int sh, int64_t nb, const uint32_t* __restrict__ counts_all,
    const uint32_t* __restrict__ dbase_all) {
    constexpr int kWaves = kThreads / 64;
    constexpr int kWaveItems = kTileItems / kWaves;
    constexpr uint32_t kNone = 0xffffffffu;
    const int64_t arr = blockIdx.y;
    const uint64_t* kin = kin_all + arr * ksi;
    uint64_t* kout = kout_all + arr * kso;
    const uint32_t* pin = pin_all ? pin_all + arr * n : nullptr;
    uint32_t* pout = pout_all + arr * n;
    const uint32_t* counts = counts_all + arr * 256 * nb;
    const uint32_t* dbase = dbase_all + arr * 256;
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t tbase[256];
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint8_t sdig[kTileItems];
    __shared__ uint64_t sval[kTileItems];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kTileItems;
    const int64_t wb = t0 + (int64_t)w * kWaveItems;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

#pragma unroll
    for (int j = 0; j < 4; j++) wcnt[w][lane + 64 * j] = 0;
    tbase[tid] = dbase[tid] + counts[(int64_t)tid * nb + blockIdx.x];

    uint64_t kv[kRounds];
    uint32_t pv[kRounds], lp[kRounds];
#pragma unroll
    for (int k = 0; k < kRounds; k++) {
        const int64_t i = wb + (int64_t)k * 64 + lane;
        const bool valid = i < n;
        kv[k] = valid ? kin[i] : 0ull;
        pv[k] = valid ? (pin ? pin[i] : (uint32_t)i) : 0u;
    }
    // ranks within the wave's quarter
#pragma unroll
    for (int k = 0; k < kRounds; k++) {
        const int64_t i = wb + (int64_t)k * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = (uint32_t)(kv[k] >> sh) & 0xffu;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bl = __ballot(on);
            peers &= on ? bl : ~bl;
        }
        const int leader = valid ? __builtin_ctzll(peers) : lane;
        uint32_t old = 0;
        if (valid && lane == leader) old = atomicAdd(&wcnt[w][d], (uint32_t)__popcll(peers));
        old = (uint32_t)__shfl((int)old, leader, 64);
        lp[k] = valid ? old + (uint32_t)__popcll(peers & lt) : kNone;
    }
    __syncthreads();
    {
        // thread tid owns digit tid: tile start by an exclusive scan of the
        // digit totals, then the per-wave offsets within the digit
        uint32_t c[kWaves], x = 0;
#pragma unroll
        for (int v = 0; v < kWaves; v++) {
            c[v] = wcnt[v][tid];
            x += c[v];
        }
        uint32_t inc = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
        for (int v = 0; v < w; v++) pre += wsum[v];
        uint32_t acc = pre + inc - x;
        tstart[tid] = acc;
#pragma unroll
        for (int v = 0; v < kWaves; v++) {
            wcnt[v][tid] = acc;
            acc += c[v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRounds; k++) {
        if (lp[k] == kNone) continue;
        const uint32_t d = (uint32_t)(kv[k] >> sh) & 0xffu;
        lp[k] += wcnt[w][d];
        sdig[lp[k]] = (uint8_t)d;
        sval[lp[k]] = kv[k];
    }
    __syncthreads();
    const int64_t tn = min((int64_t)kTileItems, n - t0);
    uint32_t gp[kRounds];
#pragma unroll
    for (int s = 0; s < kRounds; s++) {
        const int slot = s * kThreads + tid;
        gp[s] = 0;
        if (slot < tn) {
            const uint32_t d = sdig[slot];
            gp[s] = tbase[d] + (uint32_t)slot - tstart[d];
            kout[gp[s]] = sval[slot];
        }
    }
    __syncthreads();
    uint32_t* sp = reinterpret_cast<uint32_t*>(sval);
#pragma unroll
    for (int k = 0; k < kRounds; k++)
        if (lp[k] != kNone) sp[lp[k]] = pv[k];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kRounds; s++) {
        const int slot = s * kThreads + tid;
        if (slot < tn) pout[gp[s]] = sp[slot];
    }
}

// out[a * os + i] = src[a * ss + idx[a * n + i]]
template <typename T>
__global__ void gather_kernel(const T* __restrict__ src, int64_t ss, const uint32_t* __restrict__ idx,
                              T* __restrict__ out, int64_t os, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = blockIdx.y;
    out[a * os + i] = src[a * ss + idx[a * n + i]];
}

// out[a * os + i] = src[a * ss + i]
template <typename T>
__global__ void copy_kernel(const T* __restrict__ src, int64_t ss, T* __restrict__ out, int64_t os,
                            int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = blockIdx.y;
    out[a * os + i] = src[a * ss + i];
}

// OR over items of (key XOR the array's first key), per array and word: a
// block reduces its share in LDS and adds it with one atomic per word.
__global__ __launch_bounds__(256) void varying_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                      int W64, uint64_t* __restrict__ varying) {
    __shared__ uint64_t part[4];
    const int arr = blockIdx.y;
    const uint64_t* k = keys + (int64_t)arr * W64 * n;
    for (int w = 0; w < W64; w++) {
        const uint64_t k0 = k[(int64_t)w * n];
        uint64_t acc = 0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            acc |= k[(int64_t)w * n + i] ^ k0;
        for (int off = 32; off > 0; off >>= 1) acc |= (uint64_t)__shfl_xor((long long)acc, off, 64);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint64_t b = part[0] | part[1] | part[2] | part[3];
            if (b) atomicOr((unsigned long long*)&varying[arr * W64 + w], (unsigned long long)b);
        }
        __syncthreads();
    }
}

template <typename T>
sfc_status gather(const T* src, int64_t ss, const uint32_t* idx, T* out, int64_t os, int64_t n,
                  int arrays, hipStream_t st) {
    gather_kernel<T><<<dim3(blocks_for(n), arrays), 256, 0, st>>>(src, ss, idx, out, os, n);
    return launched("gather_kernel");
}

template <typename T>
sfc_status copy(const T* src, int64_t ss, T* out, int64_t os, int64_t n, int arrays,
                hipStream_t st) {
    copy_kernel<T><<<dim3(blocks_for(n), arrays), 256, 0, st>>>(src, ss, out, os, n);
    return launched("copy_kernel");
}

}  // namespace

size_t sort_scratch_bytes(int64_t n, int W64, int arrays) {
    const int64_t nb = (n + kTileItems - 1) / kTileItems;
    const size_t per_item = W64 == 1 ? 12 : 24;   // one or two (word, payload) buffers
    return (size_t)arrays * ((size_t)n * per_item + (size_t)(256 * nb + 512) * 4) + 512;
}

sfc_status launch_varying_bits(const uint64_t* keys, int64_t n, int W64, int arrays,
                               uint64_t* varying, hipStream_t st) {
    if (n == 0 || arrays == 0) return SFC_OK;
    // about 2048 workgroups in all
    const int64_t per = std::max<int64_t>(1, 2048 / arrays);
    const unsigned nb = (unsigned)std::min<int64_t>(per, (n + 255) / 256);
    varying_kernel<<<dim3(nb, arrays), 256, 0, st>>>(keys, n, W64, varying);
    return launched("varying_kernel");
}

sfc_status radix_sort(uint64_t* keys, uint32_t* ids, int64_t n, int W64, int arrays,
                      const SortPlan& plan, void* scratch, hipStream_t st) {
    if (n <= 1 || plan.n_passes == 0 || arrays == 0) return SFC_OK;
    if (W64 < 1 || W64 > kMaxKeyWords) return fail(SFC_EINVAL, "sort: bad key word count");
    const int64_t nb = (n + kTileItems - 1) / kTileItems;
    if (nb > 0x7fffffff || arrays > 65535) return fail(SFC_EUNSUPPORTED, "sort grid too large");
    const int64_t kstride = (int64_t)W64 * n;   // between arrays in keys
    char* p = static_cast<char*>(scratch);
    uint64_t* kbuf[2];
    uint32_t* pbuf[2];
    kbuf[0] = reinterpret_cast<uint64_t*>(p);
    p += (size_t)arrays * n * 8;
    kbuf[1] = W64 > 1 ? reinterpret_cast<uint64_t*>(p) : nullptr;
    if (W64 > 1) p += (size_t)arrays * n * 8;
    pbuf[0] = reinterpret_cast<uint32_t*>(p);
    p += (size_t)arrays * n * 4;
    pbuf[1] = W64 > 1 ? reinterpret_cast<uint32_t*>(p) : nullptr;
    if (W64 > 1) p += (size_t)arrays * n * 4;
    p = reinterpret_cast<char*>(((uintptr_t)p + 255) & ~uintptr_t(255));
    uint32_t* counts = reinterpret_cast<uint32_t*>(p);
    uint32_t* totals = counts + (size_t)arrays * 256 * nb;
    uint32_t* dbase = totals + (size_t)arrays * 256;

    // one pass: (kin, ksi, pin) -> (kout, kso, pout) on the digit at bit sh
    auto pass = [&](const uint64_t* kin, int64_t ksi, uint64_t* kout, int64_t kso,
                    const uint32_t* pin, uint32_t* pout, int sh) -> sfc_status {
        hist_kernel<<<dim3((unsigned)nb, arrays), kThreads, 0, st>>>(kin, ksi, n, sh, nb, counts);
        SFC_TRY(launched("hist_kernel"));
        scan_digit_kernel<<<dim3(256, arrays), kThreads, 0, st>>>(counts, nb, totals);
        SFC_TRY(launched("scan_digit_kernel"));
        digit_base_kernel<<<arrays, 64, 0, st>>>(totals, dbase);
        SFC_TRY(launched("digit_base_kernel"));
        scatter_kernel<<<dim3((unsigned)nb, arrays), kThreads, 0, st>>>(
            kin, ksi, kout, kso, pin, pout, n, sh, nb, counts, dbase);
        return launched("scatter_kernel");
    };

    // passes grouped by word; digits ascend, so words go from W64-1 down
    int npw[kMaxKeyWords] = {0};
    for (int ps = 0; ps < plan.n_passes; ps++) {
        const int w = W64 - 1 - (plan.pass_bits[ps] >> 6);
        if (w < 0 || w >= W64) return fail(SFC_EINVAL, "sort: digit outside the key");
        npw[w]++;
    }
    int nvary = 0;
    for (int w = 0; w < W64; w++) nvary += npw[w] > 0;

    if (nvary == 1) {
        // one varying word: sort (that word, id) pairs, ping-ponging between
        // the arrays themselves and scratch; the other words are constant
        // within each array and keep their values
        const int w = W64 - 1 - (plan.pass_bits[0] >> 6);
        uint64_t* kw = keys + (int64_t)w * n;
        for (int ps = 0; ps < plan.n_passes; ps++) {
            const int sh = plan.pass_bits[ps] & 63;
            if ((ps & 1) == 0) SFC_TRY(pass(kw, kstride, kbuf[0], n, ids, pbuf[0], sh));
            else SFC_TRY(pass(kbuf[0], n, kw, kstride, pbuf[0], ids, sh));
        }
        if (plan.n_passes & 1) {
            SFC_TRY(copy(kbuf[0], n, kw, kstride, n, arrays, st));
            SFC_TRY(copy(pbuf[0], n, ids, n, n, arrays, st));
        }
        return SFC_OK;
    }

    // several varying words: passes on (word, rank) pairs
    int kc = -1, pc = -1;        // buffers holding the current words / ranks
    int last = -1;               // the word sorted last
    int ps = 0;
    for (int w = W64 - 1; w >= 0; w--) {
        if (npw[w] == 0) continue;
        const uint64_t* kin;
        int64_t ksi;
        if (last < 0) {
            kin = keys + (int64_t)w * n;   // first word: rank = item index
            ksi = kstride;
        } else {
            const int kf = kc ^ 1;
            SFC_TRY(gather(keys + (int64_t)w * n, kstride, pbuf[pc], kbuf[kf], n, n, arrays, st));
            kc = kf;
            kin = kbuf[kc];
            ksi = n;
        }
        for (int j = 0; j < npw[w]; j++, ps++) {
            const int ko = (kc < 0) ? 0 : (kin == kbuf[kc] ? kc ^ 1 : kc);
            const int po = (pc < 0) ? 0 : pc ^ 1;
            SFC_TRY(pass(kin, ksi, kbuf[ko], n, pc < 0 ? nullptr : pbuf[pc], pbuf[po],
                         plan.pass_bits[ps] & 63));
            kc = ko;
            pc = po;
            kin = kbuf[kc];
            ksi = n;
        }
        last = w;
    }
    // final order: ids and the other varying words gathered by rank into the
    // free buffers, then copied back; the word sorted last is in kbuf[kc]
    const uint32_t* rank = pbuf[pc];
    SFC_TRY(gather(ids, n, rank, pbuf[pc ^ 1], n, n, arrays, st));
    for (int w = 0; w < W64; w++) {
        if (npw[w] == 0 || w == last) continue;
        SFC_TRY(gather(keys + (int64_t)w * n, kstride, rank, kbuf[kc ^ 1], n, n, arrays, st));
        SFC_TRY(copy(kbuf[kc ^ 1], n, keys + (int64_t)w * n, kstride, n, arrays, st));
    }
    SFC_TRY(copy(kbuf[kc], n, keys + (int64_t)last * n, kstride, n, arrays, st));
    SFC_TRY(copy(pbuf[pc ^ 1], n, ids, n, n, arrays, st));
    return SFC_OK;
}

}  // namespace sfc
