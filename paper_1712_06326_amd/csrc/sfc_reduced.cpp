// Host orchestration of the reduced-precision full scan: exact-integer bf16
// MFMA filter (two passes), exact rescoring of each query's candidate set,
// float32 scan for the queries the filter cannot settle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <vector>

#include "index.hpp"
#include "mfma_scan.hpp"

namespace sfc {

namespace {

__global__ void gather_queries_kernel(const float* __restrict__ t, const uint8_t* __restrict__ m,
                                      const int64_t* __restrict__ idx, int64_t nq, int64_t tw,
                                      int64_t mw, float* __restrict__ t2, uint8_t* __restrict__ m2) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nq * tw) return;
    const int64_t q = f / tw, i = f - q * tw;
    const int64_t src = idx[q];
    if (i < tw) t2[q * tw + i] = t[src * tw + i];
    if (i < mw) m2[q * mw + i] = m[src * mw + i];
}

__global__ void scatter_results_kernel(const uint64_t* __restrict__ best, const int64_t* __restrict__ idx,
                                       int64_t nq, int64_t* __restrict__ id, float* __restrict__ cost) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const uint64_t b = best[q];
    id[idx[q]] = b == ~0ull ? -1 : (int64_t)(b & 0xffffffffull);
    cost[idx[q]] = b == ~0ull ? __builtin_inff() : __uint_as_float((uint32_t)(b >> 32));
}

constexpr double kMaxOperandBytes = 32.0 * (1ull << 30);   // bf16 dictionary operand

std::atomic<int32_t> g_cap_override{0};

// candidates kept per query: 2048 .. 16384, the lists within 512 MiB
int list_capacity(int64_t Q) {
    const int32_t forced = g_cap_override.load();
    if (forced > 0) return std::max(64, forced & ~63);
    int64_t cap = (int64_t(512) << 20) / 4 / (Q > 0 ? Q : 1);
    cap = std::max<int64_t>(2048, std::min<int64_t>(16384, cap));
    return (int)(cap & ~int64_t(63));
}

}  // namespace

void set_list_capacity_override(int32_t cap) { g_cap_override.store(cap > 0 ? cap : 0); }

sfc_status query_brute_reduced(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q,
                               sfc_mode mode, int64_t* best_id, float* best_cost) {
    if (mode == SFC_MODE_BRUTE_FP8)
        return fail(SFC_EUNSUPPORTED,
                    "fp8 scan: e4m3 cannot hold byte codes exactly; use SFC_MODE_BRUTE_BF16");
    if (ix->opt.norm != SFC_NORM_L2)
        return fail(SFC_EUNSUPPORTED, "reduced-precision scan: the L1 cost is not a dot product");
    const Grid& g = ix->g;
    hipStream_t st = ix->st;
    if ((int64_t)g.Kd * g.C > 1024)
        return fail(SFC_EUNSUPPORTED, "reduced-precision scan: patch above 1024 elements");
    SFC_TRY(ensure_quantized(ix, ix->mask_copy));
    SFC_TRY(ensure_elem_offsets(ix));
    FilterArgs fa{};
    SFC_TRY(plan_filter(g.Kd, g.C, Q, ix->n, &fa));
    const int64_t Kp = fa.Kp;
    const int64_t npad = (ix->n + 255) / 256 * 256;
    if ((double)npad * Kp * 2 > kMaxOperandBytes)
        return fail(SFC_EUNSUPPORTED,
                    "reduced-precision scan: dictionary operand above 32 GiB; use SFC_MODE_BRUTE_FP32");
    if (!ix->mfma_B) {
        SFC_TRY(dev_alloc((void**)&ix->mfma_B, (size_t)npad * Kp * 2, "reduced-precision operand"));
        SFC_TRY(launch_dict_operand(ix->xq, ix->dict, ix->n, npad, ix->elem_off, g.Kd, g.C, (int)Kp,
                                    ix->mfma_B, st));
    }
    const int64_t Qpad = fa.qtiles * kFilterRows;
    const int64_t qpad_rm = scan_qpad(Q);
    const int cap = list_capacity(Q);
    // scratch layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t oA = take((size_t)Qpad * Kp * 2);
    const size_t oT2 = take((size_t)Qpad * 4), oK = take((size_t)Qpad * 4), oF = take((size_t)Qpad * 4);
    const size_t oTm = take((size_t)Q * fa.ngroups * 4);
    const size_t oThr = take((size_t)Q * 4), oCnt = take((size_t)Q * 4);
    const size_t oList = take((size_t)Q * cap * 4);
    const size_t oWork = take((size_t)fa.qtiles * fa.ctiles * 8), oNw = take(64);
    const size_t oFb = take((size_t)Q), oIdx = take((size_t)Q * 8), oN = take(64);
    const size_t oSid = take((size_t)Q * 8), oSc = take((size_t)Q * 4);
    const size_t oCs = take(compact_scratch_bytes(Q));
    SFC_TRY(ix->red.reserve(off, "reduced-precision scratch"));
    char* base = static_cast<char*>(ix->red.ptr);
    uint16_t* A = reinterpret_cast<uint16_t*>(base + oA);
    int32_t* T2 = reinterpret_cast<int32_t*>(base + oT2);
    int32_t* kq = reinterpret_cast<int32_t*>(base + oK);
    int32_t* flag = reinterpret_cast<int32_t*>(base + oF);
    int32_t* tilemin = reinterpret_cast<int32_t*>(base + oTm);
    int32_t* thr = reinterpret_cast<int32_t*>(base + oThr);
    int32_t* cnt = reinterpret_cast<int32_t*>(base + oCnt);
    uint32_t* list = reinterpret_cast<uint32_t*>(base + oList);
    uint64_t* work = reinterpret_cast<uint64_t*>(base + oWork);
    unsigned long long* nwork_dev = reinterpret_cast<unsigned long long*>(base + oNw);
    uint8_t* fb = reinterpret_cast<uint8_t*>(base + oFb);
    int64_t* fidx = reinterpret_cast<int64_t*>(base + oIdx);
    int64_t* nfb_dev = reinterpret_cast<int64_t*>(base + oN);
    void* cscratch = base + oCs;
    int64_t* seed_id = reinterpret_cast<int64_t*>(base + oSid);
    float* seed_cost = reinterpret_cast<float*>(base + oSc);

    SFC_TRY(launch_query_operand(t, m, Q, Qpad, g.Kd, g.C, (int)Kp, ix->qparams, A, T2, kq, flag,
                                 st));
    fa.A = A;
    fa.B = ix->mfma_B;
    fa.T2 = T2;
    fa.dict = ix->dict;
    fa.tilemin = tilemin;
    fa.thr = thr;
    fa.cnt = cnt;
    fa.list = list;
    fa.work = work;
    fa.cap = cap;
    if (ix->has_sfc) {
        // seeded single pass: the index answer's exact cost bounds each
        // query's optimum from above, so one GEMM pass can list every
        // candidate that may reach it
        const bool timing = ix->timer.on;
        ix->timer.on = false;
        sfc_status qs = query_index(ix, t, m, Q, seed_id, seed_cost, nullptr, nullptr);
        ix->timer.on = timing;
        SFC_TRY(qs);
        SFC_TRY(launch_seed_threshold(seed_cost, kq, flag, ix->qparams, Q, thr, st));
        SFC_TRY(ix->timer.begin("filter_kernel<list>", st));
        SFC_TRY(launch_filter_list(fa, -1, st));
        SFC_TRY(ix->timer.end(st));
        ix->last_pass1_tiles = fa.qtiles * fa.ctiles;
        ix->last_pass2_tiles = 0;
    } else {
        // two passes: per-tile minima give the threshold, then the tiles
        // that can reach it are multiplied again and listed
        SFC_TRY(ix->timer.begin("filter_kernel<min>", st));
        SFC_TRY(launch_filter_minima(fa, st));
        SFC_TRY(ix->timer.end(st));
        SFC_TRY(launch_threshold(fa, kq, flag, ix->qparams, thr, st));
        SFC_TRY(launch_select(fa, work, nwork_dev, st));
        unsigned long long nwork = 0;
        SFC_HIP(hipMemcpyAsync(&nwork, nwork_dev, sizeof(nwork), hipMemcpyDeviceToHost, st));
        SFC_HIP(hipStreamSynchronize(st));
        ix->last_pass1_tiles = fa.qtiles * fa.ctiles;
        ix->last_pass2_tiles = (int64_t)nwork;
        SFC_TRY(ix->timer.begin("filter_kernel<list>", st));
        SFC_TRY(launch_filter_list(fa, (int64_t)nwork, st));
        SFC_TRY(ix->timer.end(st));
    }
    SFC_TRY(ix->rowmask.reserve((size_t)qpad_rm * g.rows * sizeof(uint32_t), "row masks"));
    uint32_t* rm = static_cast<uint32_t*>(ix->rowmask.ptr);
    SFC_TRY(launch_pack_rowmask(m, g, Q, rm, st));
    SFC_TRY(ix->timer.begin("list_rescore_kernel", st));
    SFC_TRY(launch_list_rescore(g, ix->vol, t, rm, qpad_rm, list, cnt, thr, cap, Q, best_id,
                                best_cost, fb, SFC_NORM_L2, st));
    SFC_TRY(ix->timer.end(st));
    // queries the filter could not settle go through the float32 scan
    SFC_TRY(launch_compact(fb, Q, fidx, nullptr, Q, nfb_dev, cscratch, st));
    int64_t nfb = 0;
    SFC_HIP(hipMemcpyAsync(&nfb, nfb_dev, sizeof(nfb), hipMemcpyDeviceToHost, st));
    SFC_HIP(hipStreamSynchronize(st));
    ix->last_fallback = nfb;
    if (nfb == 0) return SFC_OK;
    const int64_t tw = (int64_t)g.Kd * g.C, mw = g.Kd;
    float* t2 = nullptr;
    uint8_t* m2 = nullptr;
    uint64_t* b2 = nullptr;
    SFC_TRY(dev_alloc((void**)&t2, (size_t)nfb * tw * 4, "fallback targets"));
    sfc_status s = dev_alloc((void**)&m2, (size_t)nfb * mw, "fallback masks");
    if (s == SFC_OK) s = dev_alloc((void**)&b2, (size_t)nfb * 8, "fallback results");
    if (s == SFC_OK) {
        gather_queries_kernel<<<(unsigned)((nfb * tw + 255) / 256), 256, 0, st>>>(
            t, m, fidx, nfb, tw, mw, t2, m2);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) s = check_hip(e, "gather_queries_kernel");
    }
    if (s == SFC_OK) s = query_brute_fp32(ix, t2, m2, nfb, b2, "scan_fp32_kernel<fallback>");
    if (s == SFC_OK) {
        scatter_results_kernel<<<(unsigned)((nfb + 255) / 256), 256, 0, st>>>(b2, fidx, nfb, best_id,
                                                                            best_cost);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) s = check_hip(e, "scatter_results_kernel");
    }
    hipError_t e = hipStreamSynchronize(st);
    dev_free(t2);
    dev_free(m2);
    dev_free(b2);
    if (s == SFC_OK && e != hipSuccess) s = check_hip(e, "fallback scan");
    return s;
}

}  // namespace sfc
