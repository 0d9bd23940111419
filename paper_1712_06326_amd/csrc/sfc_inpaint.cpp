// Host side of the fill loop: one iteration = pick the target, extract it,
// query it in the chosen mode, copy the chosen patch.
//
// Float32-scan and index modes run device-resident: the loop state (unknown
// count, target, source, iteration count) stays on the device, priorities
// are kept per voxel and recomputed only around the last filled box, and
// the iterations are replayed from HIP graphs (one of 16 iterations, one of
// 1) in rounds. A round holds floor(unknown / K^nd) iterations (at least
// one): every iteration fills at least one voxel (the target is a front
// voxel, so its box holds an unknown face neighbour) and at most K^nd, so a
// round never runs past the last iteration. The host reads the state once
// per round. The bf16 mode (whose list overflow falls back on the host)
// keeps one host round trip per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <vector>

#include "index.hpp"
#include "inpaint.hpp"

namespace sfc {

namespace {

struct DevMem {
    std::vector<void*> p;
    sfc_status alloc(void** out, size_t bytes, const char* what) {
        SFC_TRY(dev_alloc(out, bytes, what));
        p.push_back(*out);
        return SFC_OK;
    }
    ~DevMem() {
        for (void* x : p) dev_free(x);
    }
};

// Restores the handle's stream and destroys the loop's stream and graphs.
struct LoopRes {
    sfc_index* ix;
    hipStream_t saved;
    hipStream_t ls = nullptr;
    hipGraphExec_t g1 = nullptr, g16 = nullptr;
    ~LoopRes() {
        ix->st = saved;
        if (g1) (void)hipGraphExecDestroy(g1);
        if (g16) (void)hipGraphExecDestroy(g16);
        if (ls) {
            (void)hipStreamSynchronize(ls);
            (void)hipStreamDestroy(ls);
        }
    }
};

struct LoopBufs {
    float* vol;
    uint8_t* mask;
    double* conf;
    int order;
    sfc_mode mode;
    float* t;
    uint8_t* m;
    void* pv;
    void* part1;
    void* part2;
    LoopState* state;
    void* qbuf;        // query temporaries
    uint32_t* rm;      // float32 scan: row masks, padded target, packed result
    float* tp;
    uint64_t* best;
    int64_t cap;
    int64_t *lc, *ls;
    float* lcost;
};

// One iteration on the handle's stream (kernel launches only): apply the
// previous iteration's answer, refresh the priorities around it, pick and
// extract the next target, query it. With the index the query's last
// workgroup applies its answer itself, so the iteration needs no apply
// launch; the float32 scan's answer is applied at the next iteration's start.
sfc_status loop_body(sfc_index* ix, const LoopBufs& b) {
    const Grid& g = ix->g;
    hipStream_t st = ix->st;
    const bool scan = b.mode == SFC_MODE_BRUTE_FP32;
    if (scan)
        SFC_TRY(launch_loop_apply(b.vol, b.mask, b.conf, g, b.state, b.best, b.cap, b.lc, b.ls,
                                  b.lcost, st));
    SFC_TRY(launch_loop_select(b.vol, b.mask, b.conf, g, b.order, b.pv, b.part1, b.part2, b.state,
                               b.t, b.m, scan ? b.tp : nullptr, scan ? b.rm : nullptr,
                               scan_qpad(1), scan ? b.best : nullptr, st));
    if (scan) return scan_fp32_prepared(ix, 1, b.rm, b.tp, b.best);
    const LoopApply la{b.vol, b.mask, b.conf, g, b.state, b.cap, b.lc, b.ls, b.lcost};
    return query_index_on(ix, b.t, b.m, 1, b.qbuf, &b.state->source, &b.state->cost, nullptr,
                          nullptr, &la);
}

sfc_status capture(sfc_index* ix, const LoopBufs& b, int iters, hipGraphExec_t* out) {
    SFC_HIP(hipStreamBeginCapture(ix->st, hipStreamCaptureModeThreadLocal));
    sfc_status s = SFC_OK;
    for (int i = 0; i < iters && s == SFC_OK; i++) s = loop_body(ix, b);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ix->st, &graph);
    if (s != SFC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return check_hip(e, "fill loop capture");
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return check_hip(e, "fill loop graph");
    return SFC_OK;
}

}  // namespace

// The device-resident loop (float32 scan or index queries).
sfc_status device_loop(sfc_index* ix, float* volume, uint8_t* mask, double* conf, int order,
                       sfc_mode mode, float* t, uint8_t* m, int64_t cap, int64_t* lc, int64_t* lsrc,
                       float* lcost, int64_t* iters) {
    const Grid& g = ix->g;
    LoopRes res{ix, ix->st};
    SFC_HIP(hipStreamCreateWithFlags(&res.ls, hipStreamNonBlocking));
    // the loop's stream follows the work already queued on the handle's
    hipEvent_t ev = nullptr;
    SFC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t he = hipEventRecord(ev, res.saved);
    if (he == hipSuccess) he = hipStreamWaitEvent(res.ls, ev, 0);
    (void)hipEventDestroy(ev);
    if (he != hipSuccess) return check_hip(he, "fill loop stream");
    ix->st = res.ls;
    ix->timer.reset(false);

    int64_t nb1, nb2;
    loop_part_entries(g, &nb1, &nb2);
    DevMem mem;
    LoopBufs b{};
    b.vol = volume;
    b.mask = mask;
    b.conf = conf;
    b.order = order;
    b.mode = mode;
    b.t = t;
    b.m = m;
    b.cap = cap;
    b.lc = lc;
    b.ls = lsrc;
    b.lcost = lcost;
    const size_t cb = loop_cand_bytes();
    SFC_TRY(mem.alloc(&b.pv, (size_t)g.nvox * cb, "voxel priorities"));
    SFC_TRY(mem.alloc(&b.part1, (size_t)nb1 * cb, "priority partials"));
    SFC_TRY(mem.alloc(&b.part2, (size_t)nb2 * cb, "priority partials"));
    SFC_TRY(mem.alloc((void**)&b.state, sizeof(LoopState), "loop state"));
    if (mode == SFC_MODE_INDEX) {
        SFC_TRY(mem.alloc(&b.qbuf, index_query_bytes(ix, 1), "query scratch"));
    } else {
        const int64_t qpad = scan_qpad(1);
        SFC_TRY(mem.alloc((void**)&b.rm, (size_t)qpad * g.rows * 4, "row masks"));
        SFC_TRY(mem.alloc((void**)&b.tp, (size_t)qpad * g.Kd * g.C * 4, "padded target"));
        SFC_TRY(mem.alloc((void**)&b.best, 8, "scan result"));
        // query slots 1.. of the padded target and row masks stay zero
        SFC_TRY(launch_zero_f32(b.tp, qpad * g.Kd * g.C, res.ls));
        SFC_TRY(launch_zero_f32(reinterpret_cast<float*>(b.rm), qpad * g.rows, res.ls));
    }
    SFC_TRY(launch_loop_init(volume, mask, conf, g, order, b.pv, b.part1, b.part2, b.state, res.ls));

    // the first iteration runs eagerly (it also settles every lazily
    // computed launch parameter before the capture)
    SFC_TRY(loop_body(ix, b));
    SFC_TRY(capture(ix, b, 1, &res.g1));
    SFC_TRY(capture(ix, b, 16, &res.g16));
    LoopState h{};
    unsigned long long prev_unknown = ~0ull;
    const uint64_t* abest = mode == SFC_MODE_BRUTE_FP32 ? b.best : nullptr;
    for (;;) {
        // the last iteration's answer, so the unknown count is current
        SFC_TRY(launch_loop_apply(volume, mask, conf, g, b.state, abest, cap, lc, lsrc, lcost, res.ls));
        SFC_HIP(hipMemcpyAsync(&h, b.state, sizeof(h), hipMemcpyDeviceToHost, res.ls));
        SFC_HIP(hipStreamSynchronize(res.ls));
        if (h.unknown == 0) break;
        // every iteration with a target fills at least one voxel, so a whole
        // round that leaves the unknown count unchanged had no target
        if (h.unknown >= prev_unknown)
            return fail(SFC_EEMPTY, "unknown voxels remain but the fill front is empty");
        prev_unknown = h.unknown;
        int64_t r = (int64_t)(h.unknown / (unsigned long long)g.Kd);
        if (r < 1) r = 1;
        for (; r >= 16; r -= 16) SFC_HIP(hipGraphLaunch(res.g16, res.ls));
        for (; r > 0; r--) SFC_HIP(hipGraphLaunch(res.g1, res.ls));
    }
    *iters = h.it;
    return SFC_OK;
}

}  // namespace sfc

using namespace sfc;

extern "C" sfc_status sfc_inpaint(float* volume, uint8_t* mask, const sfc_geometry* g, int32_t K,
                                  sfc_order order, sfc_mode mode, sfc_index* idx,
                                  const sfc_options* opt, int64_t* n_iters, sfc_fill_log* log) {
    clear_error();
    if (!volume || !mask || !g || !n_iters) return fail(SFC_EINVAL, "sfc_inpaint: null pointer");
    if (K < 3) return fail(SFC_EINVAL, "sfc_inpaint: K must be >= 3 (a target must cover an unknown voxel)");
    if (order != SFC_ORDER_CRIMINISI && order != SFC_ORDER_RASTER) return fail(SFC_EINVAL, "unknown order");
    if (mode < SFC_MODE_BRUTE_FP32 || mode > SFC_MODE_INDEX) return fail(SFC_EINVAL, "unknown mode");
    if (log && (log->cap < 0 || (log->cap > 0 && (!log->centre_host || !log->source_host || !log->cost_host))))
        return fail(SFC_EINVAL, "sfc_inpaint: bad log");
    if ((opt && opt->struct_size > offsetof(sfc_options, norm) && opt->norm != SFC_NORM_L2) ||
        (idx && idx->opt.norm != SFC_NORM_L2))
        return fail(SFC_EUNSUPPORTED, "sfc_inpaint: the fill loop uses the L2 cost");
    sfc_index* ix = idx;
    sfc_index* owned = nullptr;
    if (!ix) {
        sfc_status s;
        if (mode == SFC_MODE_INDEX) {
            int Kd = 1;
            for (int i = 0; i < g->ndim; i++) Kd *= K;
            const int D = std::min(8, (6 * Kd + 9) / 10 * g->channels);
            s = sfc_index_build(volume, mask, g, K, D, std::min(4, D + 1), opt, &owned);
        } else {
            s = sfc_dictionary_build(volume, mask, g, K, opt, &owned);
        }
        if (s != SFC_OK) return s;
        ix = owned;
    } else {
        if (ix->vol != volume || ix->g.K != K || ix->g.nd != g->ndim || ix->g.C != g->channels)
            return fail(SFC_EINVAL, "sfc_inpaint: index was built for another volume or patch size");
        if (mode == SFC_MODE_INDEX && !ix->has_sfc)
            return fail(SFC_EINVAL, "sfc_inpaint: index mode needs an SFC index handle");
    }
    struct Free {
        sfc_index* h;
        ~Free() { sfc_index_free(h); }
    } free_owned{owned};
    const Grid& gr = ix->g;
    hipStream_t st = ix->st;
    const int64_t cap = log ? log->cap : 0;
    DevMem mem;
    double* conf = nullptr;
    void* part = nullptr;
    struct Small {
        unsigned long long unknown;
        int64_t centre;
        double cpick;
        int64_t source;
        float cost;
        float pad;
    };
    Small* sm = nullptr;
    float* t = nullptr;
    uint8_t* m = nullptr;
    int64_t *lc = nullptr, *ls = nullptr;
    float* lcost = nullptr;
    uint64_t* packed = nullptr;
    SFC_TRY(mem.alloc((void**)&conf, (size_t)gr.nvox * 8, "confidence"));
    SFC_TRY(mem.alloc(&part, inpaint_part_bytes(gr), "priority partials"));
    SFC_TRY(mem.alloc((void**)&sm, sizeof(Small), "loop state"));
    SFC_TRY(mem.alloc((void**)&t, (size_t)gr.Kd * gr.C * 4, "target"));
    SFC_TRY(mem.alloc((void**)&m, (size_t)gr.Kd, "target mask"));
    SFC_TRY(mem.alloc((void**)&packed, 8, "scan result"));
    SFC_TRY(mem.alloc((void**)&lc, (size_t)std::max<int64_t>(cap, 1) * 8, "log"));
    SFC_TRY(mem.alloc((void**)&ls, (size_t)std::max<int64_t>(cap, 1) * 8, "log"));
    SFC_TRY(mem.alloc((void**)&lcost, (size_t)std::max<int64_t>(cap, 1) * 4, "log"));
    SFC_TRY(launch_conf_init(mask, gr, conf, st));
    if (mode == SFC_MODE_BRUTE_FP32 || mode == SFC_MODE_INDEX) {
        int64_t it = 0;
        SFC_TRY(device_loop(ix, volume, mask, conf, order == SFC_ORDER_CRIMINISI ? 0 : 1, mode, t,
                            m, cap, lc, ls, lcost, &it));
        if (log) {
            const int64_t k = std::min(it, cap);
            if (k > 0) {
                SFC_HIP(hipMemcpy(log->centre_host, lc, (size_t)k * 8, hipMemcpyDeviceToHost));
                SFC_HIP(hipMemcpy(log->source_host, ls, (size_t)k * 8, hipMemcpyDeviceToHost));
                SFC_HIP(hipMemcpy(log->cost_host, lcost, (size_t)k * 4, hipMemcpyDeviceToHost));
            }
            log->len = k;
        }
        *n_iters = it;
        return SFC_OK;
    }
    int64_t it = 0;
    for (;;) {
        SFC_TRY(launch_pick(volume, mask, conf, gr, order == SFC_ORDER_CRIMINISI ? 0 : 1, part,
                            &sm->unknown, &sm->centre, &sm->cpick, st));
        Small h{};
        SFC_HIP(hipMemcpyAsync(&h, sm, sizeof(Small), hipMemcpyDeviceToHost, st));
        SFC_HIP(hipStreamSynchronize(st));
        if (h.unknown == 0) break;
        if (h.centre < 0) return fail(SFC_EEMPTY, "unknown voxels remain but the fill front is empty");
        SFC_TRY(launch_extract(volume, mask, gr, &sm->centre, 1, t, m, st));
        if (mode == SFC_MODE_BRUTE_FP32) {
            SFC_TRY(query_brute_fp32(ix, t, m, 1, packed));
            SFC_TRY(launch_unpack_best(packed, 1, &sm->source, &sm->cost, st));
        } else if (mode == SFC_MODE_INDEX) {
            SFC_TRY(query_index(ix, t, m, 1, &sm->source, &sm->cost, nullptr, nullptr));
        } else {
            SFC_TRY(query_brute_reduced(ix, t, m, 1, mode, &sm->source, &sm->cost));
        }
        SFC_TRY(launch_fill(volume, mask, conf, gr, &sm->centre, &sm->source, &sm->cost, &sm->cpick,
                            it, cap, lc, ls, lcost, st));
        it++;
    }
    if (log) {
        const int64_t k = std::min(it, cap);
        if (k > 0) {
            SFC_HIP(hipMemcpyAsync(log->centre_host, lc, (size_t)k * 8, hipMemcpyDeviceToHost, st));
            SFC_HIP(hipMemcpyAsync(log->source_host, ls, (size_t)k * 8, hipMemcpyDeviceToHost, st));
            SFC_HIP(hipMemcpyAsync(log->cost_host, lcost, (size_t)k * 4, hipMemcpyDeviceToHost, st));
        }
        log->len = k;
    }
    SFC_HIP(hipStreamSynchronize(st));
    *n_iters = it;
    return SFC_OK;
}
