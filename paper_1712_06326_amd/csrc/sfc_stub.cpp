// Temporary: SFC entry points not yet wired.
#include "index.hpp"
namespace sfc {
sfc_status check_sfc_args(const sfc_geometry*, int, int, int, const sfc_options&) { return SFC_OK; }
sfc_status build_sfc(sfc_index*, const uint8_t*, int, int, const int8_t*) { return fail(SFC_EUNSUPPORTED, "SFC index not built in this version"); }
void release_sfc(sfc_index*) {}
sfc_status query_brute_reduced(sfc_index*, const float*, const uint8_t*, int64_t, sfc_mode, int64_t*, float*) { return fail(SFC_EUNSUPPORTED, "reduced-precision scan not built"); }
sfc_status query_index(sfc_index*, const float*, const uint8_t*, int64_t, int64_t*, float*, int64_t*, int32_t*) { return fail(SFC_EUNSUPPORTED, "index query not built"); }
sfc_status query_coords(sfc_index*, const float*, const uint8_t*, int64_t, int32_t*, double*) { return fail(SFC_EUNSUPPORTED, "not built"); }
}
extern "C" {
sfc_status sfc_index_quantized(const sfc_index*, uint8_t*) { return sfc::fail(SFC_EUNSUPPORTED, "not built"); }
sfc_status sfc_index_get_basis(const sfc_index*, int32_t, int8_t*, int32_t*) { return sfc::fail(SFC_EUNSUPPORTED, "not built"); }
sfc_status sfc_index_get_params(const sfc_index*, int32_t, int64_t*, int64_t*) { return sfc::fail(SFC_EUNSUPPORTED, "not built"); }
sfc_status sfc_index_projection(const sfc_index*, int32_t, int64_t*) { return sfc::fail(SFC_EUNSUPPORTED, "not built"); }
sfc_status sfc_index_export(const sfc_index*, int32_t, int32_t, uint64_t*, int64_t*) { return sfc::fail(SFC_EUNSUPPORTED, "not built"); }
sfc_status sfc_inpaint(float*, uint8_t*, const sfc_geometry*, int32_t, sfc_order, sfc_mode, sfc_index*, const sfc_options*, int64_t*, sfc_fill_log*) { return sfc::fail(SFC_EUNSUPPORTED, "not built"); }
}
