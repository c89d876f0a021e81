// temporary: entry points not yet implemented
#include "sd_host.h"
using namespace sd;
namespace sd { void batch_release_graphs() {} }
extern "C" {
sd_status mobility_adjoint(const sd_params*, int64_t, const void*, const void*, const void*, double*, double*, int32_t, void*) { return fail(SD_EUNSUPPORTED, "not yet"); }
sd_status sd_run_adjoint(const sd_params*, int64_t, const double*, const void*, double, int64_t, int32_t, const double*, int64_t, const double*, double*, double*, void*) { return fail(SD_EUNSUPPORTED, "not yet"); }
sd_status sd_batch_create(const sd_params*, int64_t, const int64_t*, sd_batch**) { return fail(SD_EUNSUPPORTED, "not yet"); }
sd_status sd_batch_destroy(sd_batch*) { return SD_OK; }
int64_t sd_batch_particles(const sd_batch*) { return 0; }
sd_status mobility_apply_batched(sd_batch*, const void*, const void*, double*, int32_t, void*) { return fail(SD_EUNSUPPORTED, "not yet"); }
sd_status sd_run_batched(sd_batch*, double*, const void*, double, int64_t, int32_t, int32_t, int32_t, void*) { return fail(SD_EUNSUPPORTED, "not yet"); }
sd_status sd_autotune(const sd_params*, int64_t, int32_t, void*, char*, int64_t) { return fail(SD_EUNSUPPORTED, "not yet"); }
}
