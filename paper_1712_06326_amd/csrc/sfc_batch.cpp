// Batches of independent 2D images of uneven size, each with its own
// dictionary (Section I's full scan per image), answered by one persistent
// float32-scan launch over (image, query block, tile chunk) work items. The
// whole query (target packing, scan, result unpacking) is captured once in a
// HIP graph on the batch's own stream and replayed while the query layout
// (per-image counts and buffers) stays the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "batch.hpp"
#include "index.hpp"

namespace sfc {
namespace {

constexpr int kBatchShapes = 3;
constexpr int64_t kBatchQueriesPerItem = 256;
constexpr int64_t kBatchTargetItems = 16384;

int device_cus_b() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        return v;
    return 256;
}

}  // namespace
}  // namespace sfc

struct sfc_batch {
    std::vector<sfc_index*> imgs;
    int K = 0;
    hipStream_t user = nullptr;   // caller's stream (ordering only)
    hipStream_t st = nullptr;     // own non-blocking stream: capture and replay
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int shape = 0;
    // layout of the cached graph
    std::vector<int64_t> counts;
    const void *key_t = nullptr, *key_m = nullptr, *key_id = nullptr, *key_cost = nullptr;
    int key_shape = -1;
    int64_t n_items = 0;
    sfc::Scratch tables, tpad, rowmask, best;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t replays = 0;

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key_shape = -1;
    }
    ~sfc_batch() {
        drop_graph();
        for (sfc_index* h : imgs) sfc_index_free(h);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (st) (void)hipStreamDestroy(st);
    }
};

namespace sfc {
namespace {

// Tables for the current counts, then the graph that replays the query.
sfc_status build_graph(sfc_batch* b, const float* targets, const uint8_t* masks,
                       const int64_t* counts, int64_t* best_id, float* best_cost) {
    b->drop_graph();
    const int n = (int)b->imgs.size();
    const int K = b->K, Kd = K * K;
    std::vector<BatchMeta> meta(n);
    std::vector<int64_t> pad_start(n + 1, 0);
    int64_t q_off = 0, t_off = 0, tpad_off = 0, rm_off = 0;
    for (int i = 0; i < n; i++) {
        const int C = b->imgs[i]->g.C;
        BatchMeta& m = meta[i];
        m.Q = counts[i];
        m.qpad = scan_qpad(counts[i]);
        m.q_off = q_off;
        m.t_off = t_off;
        m.tpad_off = tpad_off;
        m.rm_off = rm_off;
        m.C = C;
        q_off += m.Q;
        t_off += m.Q * Kd * C;
        tpad_off += m.qpad * Kd * C;
        rm_off += m.qpad * K;
        pad_start[i + 1] = pad_start[i] + m.qpad;
    }
    const int64_t Qt = q_off, total_pad = pad_start[n];
    SFC_TRY(b->tpad.reserve((size_t)std::max<int64_t>(1, tpad_off) * 4, "batch targets"));
    SFC_TRY(b->rowmask.reserve((size_t)std::max<int64_t>(1, rm_off) * 4, "batch row masks"));
    SFC_TRY(b->best.reserve((size_t)std::max<int64_t>(1, Qt) * 8, "batch results"));
    float* tp = static_cast<float*>(b->tpad.ptr);
    uint32_t* rm = static_cast<uint32_t*>(b->rowmask.ptr);
    uint64_t* bs = static_cast<uint64_t*>(b->best.ptr);

    // per-image scan parameters and the work items
    std::vector<ScanParams> params(n);
    std::vector<int32_t> chan(n);
    std::vector<int64_t> tiles(n);
    const int qb = batch_query_block(b->shape);
    const int64_t qpw = (kBatchQueriesPerItem + qb - 1) / qb * qb;
    int64_t work = 0;
    for (int i = 0; i < n; i++) {
        const sfc_index* h = b->imgs[i];
        params[i] = batch_image_params(h->g, h->vol, h->valid, h->spans, h->n_spans,
                                       tp + meta[i].tpad_off,
                                       rm + meta[i].rm_off, bs + meta[i].q_off, meta[i].Q,
                                       meta[i].qpad, b->shape, &tiles[i]);
        chan[i] = h->g.C;
        work += ((meta[i].Q + qpw - 1) / qpw) * tiles[i];
    }
    int64_t tpw = std::max<int64_t>(4, (work + kBatchTargetItems - 1) / kBatchTargetItems);
    tpw = (tpw + 3) / 4 * 4;
    std::vector<BatchItem> items;
    for (int i = 0; i < n; i++)
        for (int64_t t0 = 0; t0 < tiles[i]; t0 += tpw)
            for (int64_t q0 = 0; q0 < meta[i].Q; q0 += qpw)
                items.push_back(BatchItem{i, 0, q0, std::min(meta[i].Q, q0 + qpw), t0,
                                          std::min(tiles[i], t0 + tpw)});
    b->n_items = (int64_t)items.size();

    // one device block for every table
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_par = 0, o_c = o_par + al(n * sizeof(ScanParams));
    const size_t o_it = o_c + al(n * sizeof(int32_t));
    const size_t o_meta = o_it + al(std::max<size_t>(1, items.size()) * sizeof(BatchItem));
    const size_t o_ps = o_meta + al(n * sizeof(BatchMeta));
    const size_t total = o_ps + al((n + 1) * sizeof(int64_t));
    SFC_TRY(b->tables.reserve(total, "batch tables"));
    char* tb = static_cast<char*>(b->tables.ptr);
    std::vector<char> host(total, 0);
    std::memcpy(host.data() + o_par, params.data(), n * sizeof(ScanParams));
    std::memcpy(host.data() + o_c, chan.data(), n * sizeof(int32_t));
    if (!items.empty()) std::memcpy(host.data() + o_it, items.data(), items.size() * sizeof(BatchItem));
    std::memcpy(host.data() + o_meta, meta.data(), n * sizeof(BatchMeta));
    std::memcpy(host.data() + o_ps, pad_start.data(), (n + 1) * sizeof(int64_t));
    SFC_HIP(hipMemcpyAsync(tb, host.data(), total, hipMemcpyHostToDevice, b->st));
    SFC_HIP(hipStreamSynchronize(b->st));

    const unsigned grid = (unsigned)std::max<int64_t>(
        8, std::min<int64_t>(b->n_items, 4 * (int64_t)device_cus_b()) / 8 * 8);
    SFC_HIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    sfc_status s = launch_batch_prep(targets, masks, reinterpret_cast<const BatchMeta*>(tb + o_meta),
                                     reinterpret_cast<const int64_t*>(tb + o_ps), n, K, total_pad,
                                     tp, rm, bs, b->st);
    if (s == SFC_OK)
        s = launch_batch_scan(K, b->shape, reinterpret_cast<const ScanParams*>(tb + o_par),
                              reinterpret_cast<const int32_t*>(tb + o_c),
                              reinterpret_cast<const BatchItem*>(tb + o_it), b->n_items, grid, b->st);
    if (s == SFC_OK) s = launch_unpack_best(bs, Qt, best_id, best_cost, b->st);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->st, &g);
    if (s != SFC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (ce != hipSuccess) return check_hip(ce, "hipStreamEndCapture");
    b->graph = g;
    SFC_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->counts.assign(counts, counts + n);
    b->key_t = targets;
    b->key_m = masks;
    b->key_id = best_id;
    b->key_cost = best_cost;
    b->key_shape = b->shape;
    return SFC_OK;
}

sfc_status run_batch(sfc_batch* b, const float* targets, const uint8_t* masks,
                     const int64_t* counts, int64_t* best_id, float* best_cost) {
    const int n = (int)b->imgs.size();
    const bool same = b->exec && b->key_shape == b->shape && b->key_t == targets &&
                      b->key_m == masks && b->key_id == best_id && b->key_cost == best_cost &&
                      std::equal(b->counts.begin(), b->counts.end(), counts) &&
                      (int)b->counts.size() == n;
    // order after the caller's stream, run, and make the caller's stream wait
    SFC_HIP(hipEventRecord(b->ev_in, b->user));
    SFC_HIP(hipStreamWaitEvent(b->st, b->ev_in, 0));
    if (!same) SFC_TRY(build_graph(b, targets, masks, counts, best_id, best_cost));
    SFC_HIP(hipGraphLaunch(b->exec, b->st));
    b->replays++;
    SFC_HIP(hipEventRecord(b->ev_out, b->st));
    SFC_HIP(hipStreamWaitEvent(b->user, b->ev_out, 0));
    return SFC_OK;
}

}  // namespace
}  // namespace sfc

using namespace sfc;

extern "C" {

sfc_status sfc_batch_create(int32_t n_images, const float* const* volumes, const uint8_t* const* masks,
                            const sfc_geometry* geoms, int32_t K, const sfc_options* opt,
                            sfc_batch** out) {
    if (!out || !volumes || !masks || !geoms) return fail(SFC_EINVAL, "sfc_batch_create: null pointer");
    if (n_images < 1) return fail(SFC_EINVAL, "sfc_batch_create: n_images must be >= 1");
    if (!batch_scan_supported(K)) return fail(SFC_EUNSUPPORTED, "batched scan: K must be 5, 7, 9 or 11");
    for (int i = 0; i < n_images; i++) {
        if (geoms[i].ndim != 2) return fail(SFC_EUNSUPPORTED, "batched scan: images must be 2D");
        if (geoms[i].channels < 1 || geoms[i].channels > 3)
            return fail(SFC_EUNSUPPORTED, "batched scan: 1 to 3 channels");
        if (!volumes[i] || !masks[i]) return fail(SFC_EINVAL, "sfc_batch_create: null image");
    }
    const sfc_options o = resolve_options(opt);
    if (o.norm != SFC_NORM_L2) return fail(SFC_EUNSUPPORTED, "batched scan: L2 cost only");
    sfc_batch* b = new sfc_batch();
    b->K = K;
    b->user = static_cast<hipStream_t>(o.stream);
    hipError_t e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete b;
        return check_hip(e, "batch stream");
    }
    for (int i = 0; i < n_images; i++) {
        sfc_index* h = nullptr;
        const sfc_status s = sfc_dictionary_build(volumes[i], masks[i], &geoms[i], K, &o, &h);
        if (s != SFC_OK) {
            delete b;
            return s;
        }
        b->imgs.push_back(h);
    }
    *out = b;
    return SFC_OK;
}

sfc_status sfc_batch_query(sfc_batch* b, const float* targets, const uint8_t* target_masks,
                           const int64_t* counts_host, int64_t* best_id, float* best_cost) {
    if (!b || !counts_host) return fail(SFC_EINVAL, "sfc_batch_query: null pointer");
    int64_t Qt = 0;
    for (size_t i = 0; i < b->imgs.size(); i++) {
        if (counts_host[i] < 0) return fail(SFC_EINVAL, "sfc_batch_query: negative count");
        Qt += counts_host[i];
    }
    if (Qt == 0) return SFC_OK;
    if (!targets || !target_masks || !best_id || !best_cost)
        return fail(SFC_EINVAL, "sfc_batch_query: null pointer");
    return run_batch(b, targets, target_masks, counts_host, best_id, best_cost);
}

sfc_status sfc_batch_autotune(sfc_batch* b, const float* targets, const uint8_t* target_masks,
                              const int64_t* counts_host, int64_t* best_id, float* best_cost,
                              int32_t* chosen_host) {
    if (!b || !counts_host || !chosen_host) return fail(SFC_EINVAL, "sfc_batch_autotune: null pointer");
    hipEvent_t e0, e1;
    SFC_HIP(hipEventCreate(&e0));
    SFC_HIP(hipEventCreate(&e1));
    int bestv = 0;
    float bestms = 0.0f;
    sfc_status s = SFC_OK;
    for (int v = 0; v < kBatchShapes && s == SFC_OK; v++) {
        b->shape = v;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && s == SFC_OK; rep++) {   // the first run builds and warms up
            s = sfc_batch_query(b, targets, target_masks, counts_host, best_id, best_cost);
            if (s != SFC_OK) break;
            hipError_t he = hipEventRecord(e0, b->st);
            if (he == hipSuccess) he = hipGraphLaunch(b->exec, b->st);
            if (he == hipSuccess) he = hipEventRecord(e1, b->st);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) s = check_hip(he, "batch autotune timing");
        }
        if (s == SFC_OK && (v == 0 || ms < bestms)) {
            bestms = ms;
            bestv = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->shape = bestv;
    if (s != SFC_OK) return s;
    *chosen_host = bestv;
    return SFC_OK;
}

sfc_status sfc_batch_stats(const sfc_batch* b, int64_t* graph_replays_host, int64_t* work_items_host,
                           int32_t* shape_host) {
    if (!b || !graph_replays_host || !work_items_host || !shape_host)
        return fail(SFC_EINVAL, "sfc_batch_stats: null pointer");
    *graph_replays_host = b->replays;
    *work_items_host = b->n_items;
    *shape_host = b->shape;
    return SFC_OK;
}

void sfc_batch_free(sfc_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->st);
    delete b;
}

}  // extern "C"
