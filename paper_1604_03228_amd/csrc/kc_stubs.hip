// kc_stubs.hip -- entry points not yet served by this build.
#include "kc_host.h"

extern "C" {
int kcenter_eim(kc_handle* h, const kc_points*, int64_t, const kc_eim_params*, int64_t*,
                int64_t*, double*, int64_t*, int64_t*, kc_eim_iter*, int32_t*, void*)
{
    return h ? h->fail(KC_EUNSUPPORTED, "eim not built") : KC_EINVAL;
}
int kcenter_batch(kc_handle* h, const kc_problem*, int32_t, void*)
{
    return h ? h->fail(KC_EUNSUPPORTED, "batch not built") : KC_EINVAL;
}
}
