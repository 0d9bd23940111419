// Host side of the fill loop: one iteration = pick the target (device),
// extract it, query it in the chosen mode, copy the chosen patch (device).
// The host only reads the unknown count and the chosen centre to decide
// whether to continue.
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

}  // namespace

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
