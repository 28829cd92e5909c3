// Serving engine: placeholder until the continuous-batching engine lands.
#include "nf_runtime.h"

namespace nf {
int serve_config(size_t, int, int) { return fail(NF_E_DEVICE, "serving engine not built"); }
int64_t serve_submit(const char*, int, int, int) { return fail(NF_E_DEVICE, "serving engine not built"); }
int serve_poll(int64_t, int32_t*, int16_t*, int, bool) { return fail(NF_E_DEVICE, "serving engine not built"); }
int serve_stats(nf_serve_stats_t*) { return fail(NF_E_DEVICE, "serving engine not built"); }
void serve_shutdown() {}
}  // namespace nf
