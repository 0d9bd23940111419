// Temporary: the fill loop entry point is not wired yet.
#include "index.hpp"
extern "C" {
sfc_status sfc_inpaint(float*, uint8_t*, const sfc_geometry*, int32_t, sfc_order, sfc_mode, sfc_index*, const sfc_options*, int64_t*, sfc_fill_log*) { return sfc::fail(SFC_EUNSUPPORTED, "not built"); }
}
