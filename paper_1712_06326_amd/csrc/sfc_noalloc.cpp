// The float32 full scan (Section I) without any device allocation, for
// callers that cannot allocate: code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc. Its row masks, padded targets and
// packed per-query results live in one fixed array of this library, a copy
// per device, instead of the handle's growable buffers. The scan itself is
// the one sfc_query runs in SFC_MODE_BRUTE_FP32, so the answers are the same
// bits.
#include <mutex>

#include "index.hpp"

namespace sfc {
int64_t scan_qpad(int64_t Q);
}

using namespace sfc;

namespace {

// Every device that runs this library holds this array until the process
// ends. Host code never passes its name to a kernel: the name is a host-side
// stand-in, and the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[SFC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

// The array's address on the current device (looked up once per device).
sfc_status scratch_on_device(int dev, uint8_t** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SFC_EUNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(SFC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SFC_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

int64_t sfc_noalloc_bytes(const sfc_index* ix, int64_t Q) {
    if (!ix || Q < 0) return -1;
    const int64_t qpad = scan_qpad(Q);
    const Grid& g = ix->g;
    return (int64_t)(round256((size_t)qpad * g.rows * sizeof(uint32_t)) +
                     round256((size_t)qpad * g.Kd * g.C * sizeof(float)) +
                     round256((size_t)qpad * sizeof(uint64_t)));
}

sfc_status sfc_query_fp32_noalloc(sfc_index* ix, const float* targets,
                                  const uint8_t* target_masks, int64_t Q, int64_t* best_id,
                                  float* best_cost) {
    clear_error();
    if (!ix) return fail(SFC_EINVAL, "index is NULL");
    if (Q < 0) return fail(SFC_EINVAL, "Q must be >= 0");
    if (Q == 0) return SFC_OK;
    if (!targets || !target_masks || !best_id || !best_cost)
        return fail(SFC_EINVAL, "sfc_query_fp32_noalloc: null pointer");
    const int64_t need = sfc_noalloc_bytes(ix, Q);
    if (need > (int64_t)SFC_NOALLOC_SCRATCH_BYTES)
        return fail(SFC_EINVAL, "sfc_query_fp32_noalloc: " + std::to_string(Q) +
                                    " queries need " + std::to_string(need) +
                                    " bytes of scratch, above the fixed " +
                                    std::to_string((long long)SFC_NOALLOC_SCRATCH_BYTES));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SFC_EDEVICE, "hipGetDevice failed");
    if (dev != ix->device)
        return fail(SFC_EINVAL, "sfc_query_fp32_noalloc: the index's device must be current");
    uint8_t* base = nullptr;
    SFC_TRY(scratch_on_device(dev, &base));
    const Grid& g = ix->g;
    const int64_t qpad = scan_qpad(Q);
    uint32_t* rm = reinterpret_cast<uint32_t*>(base);
    float* tp = reinterpret_cast<float*>(base + round256((size_t)qpad * g.rows * sizeof(uint32_t)));
    uint64_t* best = reinterpret_cast<uint64_t*>(
        reinterpret_cast<uint8_t*>(tp) + round256((size_t)qpad * g.Kd * g.C * sizeof(float)));
    ix->last_fallback = 0;
    ix->last_pass1_tiles = ix->last_pass2_tiles = 0;
    ix->timer.reset(false);   // no timing events: nothing is created here
    SFC_TRY(scan_fp32_on(ix, targets, target_masks, Q, rm, tp, best));
    return launch_unpack_best(best, Q, best_id, best_cost, ix->st);
}

}  // extern "C"
