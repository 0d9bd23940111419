// C ABI: argument checks, handle lifetime and orchestration of the kernels.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "build.hpp"
#include "common.hpp"
#include "index.hpp"

namespace sfc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

sfc_status fail(sfc_status code, const std::string& msg) {
    set_error(msg);
    return code;
}

sfc_status check_hip(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return fail(SFC_ENOMEM, m);
    return fail(SFC_EDEVICE, m);
}

// Allocation with an optional injected failure: SFC_FAULT_INJECT=alloc:<n>
// makes the n-th device allocation of the process fail, and
// sfc_debug_fail_alloc(n) the n-th one from the call on (error-path tests).
static long g_alloc_count = 0;
static std::atomic<long> g_fail_in{0};   // > 0: allocations until one fails
static bool injected_failure(long at) {
    if (at >= 0 && g_alloc_count == at) return true;
    long v = g_fail_in.load();
    while (v > 0)
        if (g_fail_in.compare_exchange_weak(v, v - 1)) return v == 1;
    return false;
}
static long fault_alloc_at() {
    static long at = -2;
    if (at == -2) {
        at = -1;
        const char* s = std::getenv("SFC_FAULT_INJECT");
        if (s && std::strncmp(s, "alloc:", 6) == 0) at = std::atol(s + 6);
    }
    return at;
}

sfc_status dev_alloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    long at = fault_alloc_at();
    g_alloc_count++;
    if (injected_failure(at))
        return fail(SFC_ENOMEM, std::string(what) + ": injected allocation failure");
    if (bytes == 0) bytes = 1;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SFC_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
    }
    return SFC_OK;
}

void dev_free(void* p) {
    if (p) (void)hipFree(p);
}

// Temporaries come from a stream-ordered pool of the library (one per
// device): hipFree waits for every stream of the device, which would make an
// index build on one stream wait for a scan running on another; hipFreeAsync
// does not. Freed memory up to kPoolKeep bytes stays in the pool for reuse.
// If the pool cannot be created the temporaries fall back to hipMalloc /
// hipFree (the same choice for every temporary of that device).
namespace {
constexpr uint64_t kPoolKeep = uint64_t(8) << 30;
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;   // device -> pool (nullptr: none)

hipMemPool_t library_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pools.find(dev);
    if (it != g_pools.end()) return it->second;
    const char* env = std::getenv("SFC_TMP_POOL");
    if (env && std::strcmp(env, "0") == 0) {   // temporaries through hipMalloc / hipFree
        g_pools[dev] = nullptr;
        return nullptr;
    }
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
        (void)hipGetLastError();
        pool = nullptr;
    } else {
        uint64_t keep = kPoolKeep;
        if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess)
            (void)hipGetLastError();
    }
    g_pools[dev] = pool;
    return pool;
}
}  // namespace

sfc_status tmp_alloc(void** p, size_t bytes, const char* what, hipStream_t st) {
    hipMemPool_t pool = library_pool();
    if (!pool) return dev_alloc(p, bytes, what);
    *p = nullptr;
    long at = fault_alloc_at();
    g_alloc_count++;
    if (injected_failure(at))
        return fail(SFC_ENOMEM, std::string(what) + ": injected allocation failure");
    if (bytes == 0) bytes = 1;
    hipError_t e = hipMallocFromPoolAsync(p, bytes, pool, st);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SFC_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
    }
    return SFC_OK;
}

void tmp_free(void* p, hipStream_t st) {
    if (!p) return;
    if (library_pool()) (void)hipFreeAsync(p, st);
    else (void)hipFree(p);
}

sfc_status Scratch::reserve(size_t bytes, const char* what) {
    if (bytes <= cap) return SFC_OK;
    dev_free(ptr);
    ptr = nullptr;
    cap = 0;
    SFC_TRY(dev_alloc(&ptr, bytes, what));
    cap = bytes;
    return SFC_OK;
}

Scratch::~Scratch() { dev_free(ptr); }

static sfc_status check_geometry(const sfc_geometry* g, int K) {
    if (!g) return fail(SFC_EINVAL, "geometry is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(SFC_EINVAL, "ndim must be 2 or 3");
    if (g->channels < 1 || g->channels > kMaxChannels)
        return fail(SFC_EINVAL, "channels must be 1..16");
    int64_t nvox = 1;
    for (int i = 0; i < g->ndim; i++) {
        if (g->shape[i] < 1) return fail(SFC_EINVAL, "shape entries must be >= 1");
        nvox *= g->shape[i];
    }
    if (nvox > (int64_t)0xffffffffLL)
        return fail(SFC_EUNSUPPORTED, "more than 2^32 voxels (ids are 32-bit inside kernels)");
    if (K >= 0) {
        if (K < 1 || (K & 1) == 0) return fail(SFC_EINVAL, "patch size K must be odd and >= 1");
        if (K > 31) return fail(SFC_EUNSUPPORTED, "patch size K above 31");
        for (int i = 0; i < g->ndim; i++)
            if (K > g->shape[i]) return fail(SFC_EINVAL, "patch size K larger than a side");
    }
    return SFC_OK;
}

sfc_status KernelTimer::begin(const char* name, hipStream_t st) {
    open = false;
    if (!on || used >= kMaxMarks) return SFC_OK;
    if (used == (int)marks.size()) {
        Mark mk;
        SFC_HIP(hipEventCreate(&mk.a));
        hipError_t e = hipEventCreate(&mk.b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(mk.a);
            return check_hip(e, "hipEventCreate");
        }
        marks.push_back(mk);
    }
    marks[used].name = name;
    SFC_HIP(hipEventRecord(marks[used].a, st));
    open = true;
    return SFC_OK;
}

sfc_status KernelTimer::end(hipStream_t st) {
    if (!open) return SFC_OK;
    open = false;
    SFC_HIP(hipEventRecord(marks[used].b, st));
    used++;
    return SFC_OK;
}

KernelTimer::~KernelTimer() {
    for (auto& mk : marks) {
        (void)hipEventDestroy(mk.a);
        (void)hipEventDestroy(mk.b);
    }
}

sfc_options resolve_options(const sfc_options* in) {
    sfc_options o;
    sfc_options_default(&o);
    if (in) {
        size_t n = in->struct_size;
        if (n > sizeof(sfc_options)) n = sizeof(sfc_options);
        if (n >= sizeof(uint32_t)) std::memcpy(&o, in, n);
        o.struct_size = sizeof(sfc_options);
    }
    return o;
}

sfc_status validate_options(const sfc_options& o) {
    if (o.key_bits < 1 || o.key_bits > 31) return fail(SFC_EINVAL, "key_bits must be 1..31");
    if (o.window < 1) return fail(SFC_EINVAL, "window must be >= 1");
    if (o.curve != SFC_CURVE_MORTON && o.curve != SFC_CURVE_HILBERT)
        return fail(SFC_EINVAL, "unknown curve");
    if (o.query_block < 0) return fail(SFC_EINVAL, "query_block must be >= 0");
    if (o.norm != SFC_NORM_L2 && o.norm != SFC_NORM_L1) return fail(SFC_EINVAL, "unknown norm");
    return SFC_OK;
}

// Process-wide memory of the autotuner's choices, per (ndim, K, C).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, int> g_tuned;

void remember_variant(int nd, int K, int C, int v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(nd, K, C)] = v;
}

int recalled_variant(int nd, int K, int C) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(nd, K, C));
    return it == g_tuned.end() ? 0 : it->second;
}

// Dictionary of a handle: validity map + ascending id list.
sfc_status build_dictionary(sfc_index* ix, const uint8_t* mask) {
    const Grid& g = ix->g;
    hipStream_t st = ix->st;
    SFC_TRY(dev_alloc((void**)&ix->valid, (size_t)g.nvox, "dictionary validity map"));
    TmpBuf tmp(st);
    SFC_TRY(tmp.alloc((size_t)g.nvox + compact_scratch_bytes(g.nvox) + 64, "dictionary scratch"));
    uint8_t* t8 = static_cast<uint8_t*>(tmp.ptr);
    SFC_TRY(launch_valid_centres(mask, g, ix->valid, t8, st));
    // count, allocate, compact
    uint8_t* after = t8 + ((g.nvox + 63) / 64) * 64;
    int64_t* count_dev = reinterpret_cast<int64_t*>(after);
    void* cscratch = after + 64;
    SFC_TRY(launch_compact(ix->valid, g.nvox, nullptr, nullptr, 0, count_dev, cscratch, st));
    int64_t n = 0;
    SFC_HIP(hipMemcpyAsync(&n, count_dev, sizeof(n), hipMemcpyDeviceToHost, st));
    SFC_HIP(hipStreamSynchronize(st));
    if (n == 0) return fail(SFC_EEMPTY, "no fully known patch: the dictionary is empty");
    ix->n = n;
    SFC_TRY(dev_alloc((void**)&ix->dict, (size_t)n * sizeof(uint32_t), "dictionary ids"));
    SFC_TRY(launch_compact(ix->valid, g.nvox, nullptr, ix->dict, n, count_dev, cscratch, st));
    // the full scan's spans: flagged, counted, compacted (the flags reuse
    // the scratch, which holds nvox bytes and there are nvox / 8 slots)
    const int64_t slots = scan_span_slots(g);
    if (slots > 0 && slots < (int64_t)0xffffffffLL) {
        SFC_TRY(launch_span_flags(g, ix->valid, t8, st));
        SFC_TRY(launch_compact(t8, slots, nullptr, nullptr, 0, count_dev, cscratch, st));
        int64_t ns = 0;
        SFC_HIP(hipMemcpyAsync(&ns, count_dev, sizeof(ns), hipMemcpyDeviceToHost, st));
        SFC_HIP(hipStreamSynchronize(st));
        if (ns > 0) {
            SFC_TRY(dev_alloc((void**)&ix->spans, (size_t)ns * sizeof(uint32_t), "scan spans"));
            SFC_TRY(launch_compact(t8, slots, nullptr, ix->spans, ns, count_dev, cscratch, st));
            ix->n_spans = ns;
        }
    }
    SFC_HIP(hipStreamSynchronize(st));
    return SFC_OK;
}

}  // namespace sfc

sfc_index::~sfc_index() {
    sfc::dev_free(valid);
    sfc::dev_free(dict);
    sfc::dev_free(spans);
    sfc::release_sfc(this);
}

namespace sfc {

sfc_status scan_fp32_prepared(sfc_index* ix, int64_t Q, const uint32_t* rm, const float* tp,
                              uint64_t* best, const char* label) {
    ScanArgs a{ix->vol, ix->valid, tp, rm, Q, best, ix->opt.query_block,
               ix->opt.scan_variant > 0 ? ix->opt.scan_variant - 1 : ix->tuned_variant,
               ix->spans, ix->n_spans, ix->opt.norm};
    SFC_TRY(ix->timer.begin(label, ix->st));
    SFC_TRY(launch_scan_fp32(ix->g, a, ix->st));
    return ix->timer.end(ix->st);
}

sfc_status scan_fp32_on(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, uint32_t* rm,
                        float* tp, uint64_t* best, const char* label) {
    const Grid& g = ix->g;
    const int64_t qpad = scan_qpad(Q);
    SFC_TRY(launch_pack_rowmask(m, g, Q, rm, ix->st));
    // targets padded with zero rows up to the scan's query block
    SFC_TRY(launch_pad_f32(t, (int64_t)Q * g.Kd * g.C, (int64_t)qpad * g.Kd * g.C, tp, ix->st));
    SFC_TRY(launch_fill_u64(best, Q, ~0ull, ix->st));
    return scan_fp32_prepared(ix, Q, rm, tp, best, label);
}

sfc_status query_brute_fp32(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q,
                            uint64_t* best_dev, const char* label) {
    const Grid& g = ix->g;
    const int64_t qpad = scan_qpad(Q);
    SFC_TRY(ix->rowmask.reserve((size_t)qpad * g.rows * sizeof(uint32_t), "row masks"));
    SFC_TRY(ix->tpad.reserve((size_t)qpad * g.Kd * g.C * sizeof(float), "padded targets"));
    return scan_fp32_on(ix, t, m, Q, static_cast<uint32_t*>(ix->rowmask.ptr),
                        static_cast<float*>(ix->tpad.ptr), best_dev, label);
}

}  // namespace sfc

using namespace sfc;

extern "C" {

int32_t sfc_abi_version(void) { return SFC_ABI_VERSION; }

void sfc_debug_fail_alloc(int64_t n) { g_fail_in.store(n > 0 ? (long)n : 0); }

void sfc_debug_list_capacity(int32_t cap) { set_list_capacity_override(cap); }

const char* sfc_last_error(void) { return g_last_error.c_str(); }

void sfc_options_default(sfc_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(sfc_options);
    o->key_bits = 8;
    o->window = 32;
    o->curve = SFC_CURVE_MORTON;
    o->query_block = 0;
    o->stream = nullptr;
}

sfc_status sfc_fill_front(const uint8_t* mask, const sfc_geometry* g, int64_t* centres,
                          int64_t capacity, int64_t* count_host, void* stream) {
    clear_error();
    SFC_TRY(check_geometry(g, -1));
    if (!mask || !count_host || (capacity > 0 && !centres) || capacity < 0)
        return fail(SFC_EINVAL, "sfc_fill_front: null pointer or negative capacity");
    Grid gr = make_grid(g, 1);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch tmp;
    SFC_TRY(tmp.reserve((size_t)gr.nvox + 64 + compact_scratch_bytes(gr.nvox), "front scratch"));
    uint8_t* flags = static_cast<uint8_t*>(tmp.ptr);
    uint8_t* after = flags + ((gr.nvox + 63) / 64) * 64;
    int64_t* count_dev = reinterpret_cast<int64_t*>(after);
    SFC_TRY(launch_front_flags(mask, gr, flags, st));
    SFC_TRY(launch_compact(flags, gr.nvox, centres ? centres : count_dev, nullptr, capacity,
                           count_dev, after + 64, st));
    int64_t n = 0;
    SFC_HIP(hipMemcpyAsync(&n, count_dev, sizeof(n), hipMemcpyDeviceToHost, st));
    SFC_HIP(hipStreamSynchronize(st));
    *count_host = n;
    return SFC_OK;
}

sfc_status sfc_extract_targets(const float* volume, const uint8_t* mask, const sfc_geometry* g,
                               int32_t K, const int64_t* centres, int64_t Q, float* targets,
                               uint8_t* target_masks, void* stream) {
    clear_error();
    SFC_TRY(check_geometry(g, K));
    if (Q < 0) return fail(SFC_EINVAL, "Q must be >= 0");
    if (Q == 0) return SFC_OK;
    if (!volume || !mask || !centres || !targets || !target_masks)
        return fail(SFC_EINVAL, "sfc_extract_targets: null pointer");
    Grid gr = make_grid(g, K);
    return launch_extract(volume, mask, gr, centres, Q, targets, target_masks,
                          static_cast<hipStream_t>(stream));
}

static sfc_status new_handle(const float* volume, const uint8_t* mask, const sfc_geometry* g,
                             int32_t K, const sfc_options* opt, sfc_index** out) {
    if (!out) return fail(SFC_EINVAL, "out is NULL");
    *out = nullptr;
    SFC_TRY(check_geometry(g, K));
    if (!volume || !mask) return fail(SFC_EINVAL, "volume or mask is NULL");
    sfc_options o = resolve_options(opt);
    SFC_TRY(validate_options(o));
    sfc_index* ix = new sfc_index();
    if (hipGetDevice(&ix->device) != hipSuccess) {
        delete ix;
        return fail(SFC_EDEVICE, "hipGetDevice failed");
    }
    ix->g = make_grid(g, K);
    ix->tuned_variant = recalled_variant(g->ndim, K, g->channels);
    ix->opt = o;
    ix->st = static_cast<hipStream_t>(o.stream);
    ix->vol = volume;
    sfc_status s = dev_alloc((void**)&ix->mask_copy, (size_t)ix->g.nvox, "mask copy");
    if (s == SFC_OK) {
        hipError_t e = hipMemcpyAsync(ix->mask_copy, mask, (size_t)ix->g.nvox,
                                      hipMemcpyDeviceToDevice, ix->st);
        if (e != hipSuccess) s = check_hip(e, "mask copy");
    }
    if (s == SFC_OK) s = build_dictionary(ix, mask);
    if (s != SFC_OK) {
        delete ix;
        return s;
    }
    *out = ix;
    return SFC_OK;
}

sfc_status sfc_dictionary_build(const float* volume, const uint8_t* mask, const sfc_geometry* g,
                                int32_t K, const sfc_options* opt, sfc_index** out) {
    clear_error();
    return new_handle(volume, mask, g, K, opt, out);
}

sfc_status sfc_index_build(const float* volume, const uint8_t* mask, const sfc_geometry* g,
                           int32_t K, int32_t reduced_dim, int32_t n_curves,
                           const sfc_options* opt, sfc_index** out) {
    return sfc_index_build_with_basis(volume, mask, g, K, reduced_dim, n_curves, opt, nullptr,
                                      out);
}

sfc_status sfc_index_build_with_basis(const float* volume, const uint8_t* mask,
                                      const sfc_geometry* g, int32_t K, int32_t reduced_dim,
                                      int32_t n_curves, const sfc_options* opt,
                                      const int8_t* bases_host, sfc_index** out) {
    clear_error();
    if (!out) return fail(SFC_EINVAL, "out is NULL");
    *out = nullptr;
    SFC_TRY(check_geometry(g, K));
    sfc_options o = resolve_options(opt);
    SFC_TRY(validate_options(o));
    SFC_TRY(check_sfc_args(g, K, reduced_dim, n_curves, o));
    sfc_index* ix = nullptr;
    SFC_TRY(new_handle(volume, mask, g, K, opt, &ix));
    sfc_status s = build_sfc(ix, mask, reduced_dim, n_curves, bases_host);
    if (s != SFC_OK) {
        delete ix;
        return s;
    }
    *out = ix;
    return SFC_OK;
}

// ---- saved indices (reuse of an index built once; Section III's
// precomputed indices for dictionaries used again)
extern "C++" {
namespace {
struct IndexFileHeader {
    char magic[8];        // "SFCINDEX"
    uint32_t version;     // 1
    int32_t nd, C, K, D, L, b, curve, window, W64, S, mmax, pad[2];
    int64_t shape[3], n, nsub, R;
    float vmin, qscale;
    uint64_t dict_hash;   // FNV-1a over the dictionary ids
    uint64_t code_hash;   // checksum of the known voxels' byte codes
};
static_assert(sizeof(IndexFileHeader) == 136, "index file header has no implicit padding");
constexpr char kIndexMagic[8] = {'S', 'F', 'C', 'I', 'N', 'D', 'E', 'X'};

uint64_t fnv1a(const std::vector<uint32_t>& v) {
    uint64_t h = 1469598103934665603ull;
    for (uint32_t x : v)
        for (int k = 0; k < 4; k++) {
            h ^= (x >> (8 * k)) & 0xffu;
            h *= 1099511628211ull;
        }
    return h;
}

template <typename T>
sfc_status fetch(std::vector<T>& h, const void* d, size_t count, hipStream_t st) {
    h.resize(count);
    if (count) {
        hipError_t e = hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return check_hip(e, "index copy to the host");
    }
    return SFC_OK;
}

struct File {
    FILE* f = nullptr;
    ~File() {
        if (f) std::fclose(f);
    }
};

template <typename T>
bool put(FILE* f, const std::vector<T>& v) {
    return v.empty() || std::fwrite(v.data(), sizeof(T), v.size(), f) == v.size();
}
template <typename T>
bool get(FILE* f, std::vector<T>& v, size_t count) {
    v.resize(count);
    return count == 0 || std::fread(v.data(), sizeof(T), count, f) == count;
}
}  // namespace
}  // extern "C++"

sfc_status sfc_index_save(const sfc_index* ix, const char* path) {
    clear_error();
    if (!ix || !path) return fail(SFC_EINVAL, "sfc_index_save: null pointer");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "sfc_index_save: a dictionary-only handle has no index");
    const Grid& g = ix->g;
    const size_t P = (size_t)g.Kd * g.C, S = ix->S, n = (size_t)ix->n;
    IndexFileHeader h{};
    std::memcpy(h.magic, kIndexMagic, 8);
    h.version = 1;
    h.nd = g.nd;
    h.C = g.C;
    h.K = g.K;
    h.D = ix->D;
    h.L = ix->L;
    h.b = ix->b;
    h.curve = ix->opt.curve;
    h.window = ix->opt.window;
    h.W64 = ix->W64;
    h.S = ix->S;
    h.mmax = ix->mmax;
    for (int i = 0; i < g.nd; i++) h.shape[i] = g.shape[i];
    h.n = ix->n;
    h.nsub = ix->nsub;
    h.R = ix->R;
    h.vmin = ix->vmin;
    h.qscale = ix->qscale;
    std::vector<uint64_t> sum;
    std::vector<int8_t> basis;
    std::vector<int64_t> lo, span;
    std::vector<uint32_t> dict;
    hipStream_t st = ix->st;
    SFC_TRY(fetch(sum, ix->sum, P, st));
    SFC_TRY(fetch(basis, ix->basis, S * ix->mmax * ix->D, st));
    SFC_TRY(fetch(lo, ix->lo, S * ix->D, st));
    SFC_TRY(fetch(span, ix->span, S, st));
    SFC_TRY(fetch(dict, ix->dict, n, st));
    SFC_HIP(hipStreamSynchronize(st));
    h.dict_hash = fnv1a(dict);
    SFC_TRY(code_checksum(const_cast<sfc_index*>(ix), &h.code_hash));
    File file;
    file.f = std::fopen(path, "wb");
    if (!file.f) return fail(SFC_EINVAL, std::string("sfc_index_save: cannot open ") + path);
    const bool ok = std::fwrite(&h, sizeof(h), 1, file.f) == 1 && put(file.f, sum) &&
                    put(file.f, basis) && put(file.f, lo) && put(file.f, span);
    const bool closed = std::fclose(file.f) == 0;
    file.f = nullptr;
    if (!ok || !closed) return fail(SFC_EINVAL, std::string("sfc_index_save: write failed: ") + path);
    return SFC_OK;
}

sfc_status sfc_index_load(const float* volume, const uint8_t* mask, const sfc_geometry* g,
                          int32_t K, const sfc_options* opt, const char* path, sfc_index** out) {
    clear_error();
    if (!out || !path) return fail(SFC_EINVAL, "sfc_index_load: null pointer");
    *out = nullptr;
    SFC_TRY(check_geometry(g, K));
    File file;
    file.f = std::fopen(path, "rb");
    if (!file.f) return fail(SFC_EINVAL, std::string("sfc_index_load: cannot open ") + path);
    IndexFileHeader h{};
    if (std::fread(&h, sizeof(h), 1, file.f) != 1 || std::memcmp(h.magic, kIndexMagic, 8) != 0 ||
        h.version != 1)
        return fail(SFC_EINVAL, "sfc_index_load: not an index file of this version");
    bool same = h.nd == g->ndim && h.C == g->channels && h.K == K;
    for (int i = 0; same && i < g->ndim; i++) same = h.shape[i] == g->shape[i];
    if (!same) return fail(SFC_EINVAL, "sfc_index_load: the file was saved for another geometry or K");
    sfc_options o = resolve_options(opt);
    o.key_bits = h.b;
    o.curve = h.curve;
    o.window = h.window;
    SFC_TRY(validate_options(o));
    SFC_TRY(check_sfc_args(g, K, h.D, h.L, o));
    // bounds before any array is sized from the header: at most 3^nd - 1
    // subsets of at most kMaxSubsetElems elements
    const int max_subsets = h.nd == 2 ? 8 : 26;
    if (h.n < 1 || h.S < 1 || h.S > max_subsets || h.mmax < 1 || h.mmax > kMaxSubsetElems ||
        h.W64 != (h.D * h.b + 63) / 64)
        return fail(SFC_EINVAL, "sfc_index_load: inconsistent header");
    SavedIndex sv;
    sv.nsub = h.nsub;
    sv.vmin = h.vmin;
    sv.qscale = h.qscale;
    const size_t P = (size_t)h.C;
    size_t Kd = 1;
    for (int i = 0; i < h.nd; i++) Kd *= (size_t)K;
    const size_t S = h.S, n = (size_t)h.n;
    const bool ok = get(file.f, sv.sum, Kd * P) && get(file.f, sv.basis, S * h.mmax * h.D) &&
                    get(file.f, sv.lo, S * h.D) && get(file.f, sv.span, S);
    if (!ok) return fail(SFC_EINVAL, "sfc_index_load: the file is truncated");
    if (std::fgetc(file.f) != EOF) return fail(SFC_EINVAL, "sfc_index_load: data after the index");
    sfc_index* ix = nullptr;
    SFC_TRY(new_handle(volume, mask, g, K, &o, &ix));
    sfc_status s = SFC_OK;
    if (ix->n != h.n) s = fail(SFC_EINVAL, "index file was made from another volume or mask");
    if (s == SFC_OK) {
        std::vector<uint32_t> dict;
        s = fetch(dict, ix->dict, n, ix->st);
        if (s == SFC_OK) {
            hipError_t e = hipStreamSynchronize(ix->st);
            if (e != hipSuccess) s = check_hip(e, "dictionary copy");
        }
        if (s == SFC_OK && fnv1a(dict) != h.dict_hash)
            s = fail(SFC_EINVAL, "index file was made from another volume or mask");
    }
    uint64_t codes = 0;
    if (s == SFC_OK) s = code_checksum(ix, &codes);
    if (s == SFC_OK && codes != h.code_hash)
        s = fail(SFC_EINVAL, "index file was made from another volume or mask");
    if (s == SFC_OK) s = build_sfc(ix, mask, h.D, h.L, nullptr, &sv);
    if (s == SFC_OK && (ix->W64 != h.W64 || ix->R != h.R || ix->S != h.S || ix->mmax != h.mmax))
        s = fail(SFC_EINVAL, "sfc_index_load: the file does not match this build's index layout");
    if (s != SFC_OK) {
        delete ix;
        return s;
    }
    *out = ix;
    return SFC_OK;
}

void sfc_index_free(sfc_index* idx) { delete idx; }

sfc_status sfc_index_info_get(const sfc_index* ix, sfc_index_info* info) {
    clear_error();
    if (!ix || !info) return fail(SFC_EINVAL, "null pointer");
    std::memset(info, 0, sizeof(*info));
    info->n = ix->n;
    info->ndim = ix->g.nd;
    info->channels = ix->g.C;
    info->K = ix->g.K;
    info->P = ix->g.Kd * ix->g.C;
    info->has_sfc = ix->has_sfc ? 1 : 0;
    info->window = ix->opt.window;
    info->curve = ix->opt.curve;
    info->key_bits = ix->opt.key_bits;
    if (ix->has_sfc) {
        info->n_sub = ix->nsub;
        info->n_subsets = ix->S;
        info->reduced_dim = ix->D;
        info->n_curves = ix->L;
        info->key_words = ix->W64;
        info->vmin = ix->vmin;
        info->qscale = ix->qscale;
    }
    return SFC_OK;
}

sfc_status sfc_index_dictionary(const sfc_index* ix, int64_t* ids) {
    clear_error();
    if (!ix || !ids) return fail(SFC_EINVAL, "null pointer");
    return launch_u32_to_i64(ix->dict, ids, ix->n, ix->st);
}

sfc_status sfc_query(sfc_index* ix, const float* targets, const uint8_t* target_masks, int64_t Q,
                     sfc_mode mode, int64_t* best_id, float* best_cost) {
    clear_error();
    if (!ix) return fail(SFC_EINVAL, "index is NULL");
    if (Q < 0) return fail(SFC_EINVAL, "Q must be >= 0");
    if (Q == 0) return SFC_OK;
    if (!targets || !target_masks || !best_id || !best_cost)
        return fail(SFC_EINVAL, "sfc_query: null pointer");
    ix->last_fallback = 0;
    ix->last_pass1_tiles = ix->last_pass2_tiles = 0;
    ix->timer.reset(ix->opt.timing != 0);
    switch (mode) {
    case SFC_MODE_BRUTE_FP32: {
        SFC_TRY(ix->best.reserve((size_t)Q * sizeof(uint64_t), "query results"));
        uint64_t* best = static_cast<uint64_t*>(ix->best.ptr);
        SFC_TRY(query_brute_fp32(ix, targets, target_masks, Q, best));
        return launch_unpack_best(best, Q, best_id, best_cost, ix->st);
    }
    case SFC_MODE_BRUTE_BF16:
    case SFC_MODE_BRUTE_FP8:
        return query_brute_reduced(ix, targets, target_masks, Q, mode, best_id, best_cost);
    case SFC_MODE_INDEX:
        if (!ix->has_sfc) return fail(SFC_EINVAL, "index mode needs an SFC index handle");
        return query_index(ix, targets, target_masks, Q, best_id, best_cost, nullptr, nullptr);
    default:
        return fail(SFC_EINVAL, "unknown mode");
    }
}

sfc_status sfc_query_candidates(sfc_index* ix, const float* targets, const uint8_t* target_masks,
                                int64_t Q, int64_t* cand, int32_t* ncand) {
    clear_error();
    if (!ix) return fail(SFC_EINVAL, "index is NULL");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "candidates need an SFC index handle");
    if (Q < 0) return fail(SFC_EINVAL, "Q must be >= 0");
    if (Q == 0) return SFC_OK;
    if (!targets || !target_masks || !cand || !ncand)
        return fail(SFC_EINVAL, "sfc_query_candidates: null pointer");
    return query_index(ix, targets, target_masks, Q, nullptr, nullptr, cand, ncand);
}

sfc_status sfc_query_knn(sfc_index* ix, const float* targets, const uint8_t* target_masks,
                         int64_t Q, int32_t k, int32_t mu, int64_t* best_id, float* best_cost,
                         int64_t* cand, int32_t* ncand) {
    clear_error();
    if (!ix) return fail(SFC_EINVAL, "index is NULL");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "k-NN queries need an SFC index handle");
    if (Q < 0) return fail(SFC_EINVAL, "Q must be >= 0");
    if (k < 1 || k > 256) return fail(SFC_EINVAL, "k must be 1..256");
    if (mu < 1) return fail(SFC_EINVAL, "mu must be >= 1");
    if (ix->opt.curve != SFC_CURVE_MORTON)
        return fail(SFC_EUNSUPPORTED, "k-NN queries need Morton curves (litmax/bigmin)");
    {
        // squared cell distances are summed in int64: D * (2^b)^2 must stay
        // below 2^62
        int lg = 0;
        while ((1 << lg) < ix->D) lg++;
        if (2 * ix->b + lg > 62)
            return fail(SFC_EUNSUPPORTED,
                        "k-NN queries need 2*key_bits + ceil(log2(reduced_dim)) <= 62");
    }
    if (Q == 0) return SFC_OK;
    if (!targets || !target_masks || !best_id || !best_cost)
        return fail(SFC_EINVAL, "sfc_query_knn: null pointer");
    ix->timer.reset(ix->opt.timing != 0);
    return query_knn(ix, targets, target_masks, Q, k, mu, best_id, best_cost, cand, ncand);
}

sfc_status sfc_query_coords(sfc_index* ix, const float* targets, const uint8_t* target_masks,
                            int64_t Q, int32_t* subset, double* coords) {
    clear_error();
    if (!ix) return fail(SFC_EINVAL, "index is NULL");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "coordinates need an SFC index handle");
    if (Q < 0) return fail(SFC_EINVAL, "Q must be >= 0");
    if (Q == 0) return SFC_OK;
    if (!targets || !target_masks || !subset || !coords)
        return fail(SFC_EINVAL, "sfc_query_coords: null pointer");
    return query_coords(ix, targets, target_masks, Q, subset, coords);
}

sfc_status sfc_autotune(sfc_index* ix, const float* targets, const uint8_t* target_masks,
                        int64_t Q, int32_t* chosen) {
    clear_error();
    if (!ix || !targets || !target_masks || !chosen) return fail(SFC_EINVAL, "null pointer");
    if (Q < 1) return fail(SFC_EINVAL, "autotuning needs Q >= 1");
    if (ix->opt.norm != SFC_NORM_L2)
        return fail(SFC_EUNSUPPORTED, "autotuning: the L1 scan has one tile shape");
    const Grid& g = ix->g;
    const int nv = scan_variants(g.nd, g.K, g.C);
    if (nv == 0) return fail(SFC_EUNSUPPORTED, "no float32 scan for this shape");
    SFC_TRY(ix->best.reserve((size_t)Q * sizeof(uint64_t), "query results"));
    uint64_t* best = static_cast<uint64_t*>(ix->best.ptr);
    hipEvent_t e0, e1;
    SFC_HIP(hipEventCreate(&e0));
    SFC_HIP(hipEventCreate(&e1));
    ix->timer.reset(false);
    const int saved = ix->tuned_variant, saved_opt = ix->opt.scan_variant;
    ix->opt.scan_variant = 0;
    int bestv = 0;
    float bestms = 0.0f;
    sfc_status st = SFC_OK;
    for (int v = 0; v < nv && st == SFC_OK; v++) {
        ix->tuned_variant = v;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && st == SFC_OK; rep++) {   // first run warms up
            hipError_t he = hipEventRecord(e0, ix->st);
            if (he == hipSuccess) st = query_brute_fp32(ix, targets, target_masks, Q, best);
            if (st == SFC_OK && he == hipSuccess) he = hipEventRecord(e1, ix->st);
            if (st == SFC_OK && he == hipSuccess) he = hipEventSynchronize(e1);
            if (st == SFC_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (st == SFC_OK && he != hipSuccess) st = check_hip(he, "autotune timing");
        }
        if (st == SFC_OK && (v == 0 || ms < bestms)) {
            bestms = ms;
            bestv = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ix->opt.scan_variant = saved_opt;
    if (st != SFC_OK) {
        ix->tuned_variant = saved;
        return st;
    }
    ix->tuned_variant = bestv;
    remember_variant(g.nd, g.K, g.C, bestv);
    *chosen = bestv + 1;
    return SFC_OK;
}

sfc_status sfc_sort_pairs(uint64_t* keys, uint32_t* ids, int64_t n, int32_t key_words,
                          int32_t arrays, void* stream) {
    clear_error();
    if (!keys || !ids) return fail(SFC_EINVAL, "sfc_sort_pairs: null pointer");
    if (n < 0 || arrays < 1 || key_words < 1 || key_words > kMaxKeyWords)
        return fail(SFC_EINVAL, "sfc_sort_pairs: n < 0, arrays < 1 or key_words outside 1..4");
    if (n >= (int64_t(1) << 32)) return fail(SFC_EUNSUPPORTED, "sfc_sort_pairs: n >= 2^32");
    if (n <= 1) return SFC_OK;
    return sort_key_arrays(keys, ids, n, key_words, arrays, 64 * key_words,
                           static_cast<hipStream_t>(stream));
}

sfc_status sfc_autotune_window(sfc_index* ix, const float* targets, const uint8_t* target_masks,
                               int64_t Q, float target_recall, float max_accel_error,
                               sfc_window_trial* trials, int32_t capacity, int32_t* count,
                               int32_t* window) {
    clear_error();
    if (!ix || !targets || !target_masks || !count || !window || (capacity > 0 && !trials))
        return fail(SFC_EINVAL, "null pointer");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "window autotuning needs an SFC index handle");
    if (Q < 1) return fail(SFC_EINVAL, "window autotuning needs Q >= 1");
    if (!(target_recall >= 0.0f && target_recall <= 1.0f))
        return fail(SFC_EINVAL, "target_recall must be in [0, 1]");
    if (std::isnan(max_accel_error)) return fail(SFC_EINVAL, "max_accel_error is NaN");
    ix->timer.reset(false);
    const int saved = ix->opt.window;
    std::vector<int64_t> ref_id(Q), got_id(Q);
    std::vector<float> ref_cost(Q), got_cost(Q);
    int64_t* d_id = nullptr;
    float* d_cost = nullptr;
    SFC_TRY(dev_alloc((void**)&d_id, (size_t)Q * 8, "autotune ids"));
    sfc_status s = dev_alloc((void**)&d_cost, (size_t)Q * 4, "autotune costs");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s == SFC_OK) {
        hipError_t he = hipEventCreate(&e0);
        if (he == hipSuccess) he = hipEventCreate(&e1);
        if (he != hipSuccess) s = check_hip(he, "hipEventCreate");
    }
    // reference: the float32 full scan
    if (s == SFC_OK) {
        s = ix->best.reserve((size_t)Q * sizeof(uint64_t), "query results");
        if (s == SFC_OK) s = query_brute_fp32(ix, targets, target_masks, Q, static_cast<uint64_t*>(ix->best.ptr));
        if (s == SFC_OK) s = launch_unpack_best(static_cast<uint64_t*>(ix->best.ptr), Q, d_id, d_cost, ix->st);
        if (s == SFC_OK) {
            hipError_t he = hipMemcpyAsync(ref_id.data(), d_id, (size_t)Q * 8, hipMemcpyDeviceToHost, ix->st);
            if (he == hipSuccess) he = hipMemcpyAsync(ref_cost.data(), d_cost, (size_t)Q * 4, hipMemcpyDeviceToHost, ix->st);
            if (he == hipSuccess) he = hipStreamSynchronize(ix->st);
            if (he != hipSuccess) s = check_hip(he, "autotune reference");
        }
    }
    static const int kWindows[] = {2,  4,  6,   8,   12,  16,  24,  32,  48,
                                   64, 96, 128, 192, 256, 384, 512, 768, 1024};
    int best_w = -1, largest = -1, n_trials = 0;
    float best_recall = 0.0f, largest_recall = 0.0f;
    for (int w : kWindows) {
        if (s != SFC_OK) break;
        if ((int64_t)ix->L * w > 2048) break;
        ix->opt.window = w;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && s == SFC_OK; rep++) {   // the first run warms up
            hipError_t he = hipEventRecord(e0, ix->st);
            if (he == hipSuccess) s = query_index(ix, targets, target_masks, Q, d_id, d_cost, nullptr, nullptr);
            if (s == SFC_OK && he == hipSuccess) he = hipEventRecord(e1, ix->st);
            if (s == SFC_OK && he == hipSuccess) he = hipEventSynchronize(e1);
            if (s == SFC_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (s == SFC_OK && he != hipSuccess) s = check_hip(he, "autotune timing");
        }
        if (s != SFC_OK) break;
        hipError_t he = hipMemcpyAsync(got_id.data(), d_id, (size_t)Q * 8, hipMemcpyDeviceToHost, ix->st);
        if (he == hipSuccess) he = hipMemcpyAsync(got_cost.data(), d_cost, (size_t)Q * 4, hipMemcpyDeviceToHost, ix->st);
        if (he == hipSuccess) he = hipStreamSynchronize(ix->st);
        if (he != hipSuccess) {
            s = check_hip(he, "autotune results");
            break;
        }
        int64_t hits = 0, nz = 0;
        double ae = 0.0;
        for (int64_t q = 0; q < Q; q++) {
            hits += got_id[q] == ref_id[q];
            if (ref_cost[q] > 0.0f) {
                // the ratio of the patch distances: the L2 cost is a squared norm
                ae += (ix->opt.norm == SFC_NORM_L1
                           ? (double)got_cost[q] / (double)ref_cost[q]
                           : std::sqrt((double)got_cost[q]) / std::sqrt((double)ref_cost[q])) -
                      1.0;
                nz++;
            }
        }
        const float recall = (float)hits / (float)Q;
        const float mean_ae = nz ? (float)(ae / nz) : 0.0f;
        if (n_trials < capacity) trials[n_trials] = sfc_window_trial{w, recall, mean_ae, ms};
        n_trials++;
        largest = w;
        largest_recall = recall;
        if (best_w < 0 && recall >= target_recall &&
            (max_accel_error < 0.0f || mean_ae <= max_accel_error)) {
            best_w = w;
            best_recall = recall;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(d_id);
    dev_free(d_cost);
    if (s != SFC_OK || largest < 0) {
        ix->opt.window = saved;
        return s != SFC_OK ? s : fail(SFC_EUNSUPPORTED, "no window fits n_curves * window <= 2048");
    }
    if (best_w < 0) {
        best_w = largest;
        best_recall = largest_recall;
    }
    (void)best_recall;
    ix->opt.window = best_w;
    *window = best_w;
    *count = n_trials;
    return SFC_OK;
}

sfc_status sfc_set_timing(sfc_index* ix, int32_t on) {
    clear_error();
    if (!ix) return fail(SFC_EINVAL, "index is NULL");
    ix->opt.timing = on ? 1 : 0;
    return SFC_OK;
}

sfc_status sfc_query_stats(const sfc_index* ix, int64_t* n_fallback) {
    clear_error();
    if (!ix || !n_fallback) return fail(SFC_EINVAL, "null pointer");
    *n_fallback = ix->last_fallback;
    return SFC_OK;
}

sfc_status sfc_query_filter_tiles(const sfc_index* ix, int64_t* pass1, int64_t* pass2) {
    clear_error();
    if (!ix || !pass1 || !pass2) return fail(SFC_EINVAL, "null pointer");
    *pass1 = ix->last_pass1_tiles;
    *pass2 = ix->last_pass2_tiles;
    return SFC_OK;
}

sfc_status sfc_query_kernel_times(const sfc_index* ix, sfc_kernel_time* times, int32_t capacity,
                                  int32_t* count) {
    clear_error();
    if (!ix || !count || (capacity > 0 && !times)) return fail(SFC_EINVAL, "null pointer");
    if (capacity < 0) return fail(SFC_EINVAL, "capacity must be >= 0");
    const KernelTimer& tm = ix->timer;
    std::vector<sfc_kernel_time> out;
    for (int i = 0; i < tm.used; i++) {
        const KernelTimer::Mark& mk = tm.marks[i];
        SFC_HIP(hipEventSynchronize(mk.b));
        float ms = 0.0f;
        SFC_HIP(hipEventElapsedTime(&ms, mk.a, mk.b));
        size_t k = 0;
        while (k < out.size() && std::strcmp(out[k].kernel, mk.name) != 0) k++;
        if (k == out.size()) out.push_back(sfc_kernel_time{mk.name, 0, 0.0f});
        out[k].launches++;
        out[k].ms += ms;
    }
    for (size_t k = 0; k < out.size() && (int32_t)k < capacity; k++) times[k] = out[k];
    *count = (int32_t)out.size();
    tm.used = 0;   // read: the next queries start a new record
    return SFC_OK;
}

}  // extern "C"
