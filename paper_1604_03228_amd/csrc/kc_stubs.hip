// kc_stubs.hip -- entry points not yet served by this build.
#include "kc_host.h"

int kc_gonzalez_bf16(kc_handle* h, const kc_points*, int64_t, int64_t, int64_t*, double*,
                     int64_t*, hipStream_t)
{
    return h->fail(KC_EUNSUPPORTED, "BF16 path not built");
}

extern "C" {
int kcenter_mrg(kc_handle* h, const kc_points*, const int64_t*, int32_t, int64_t, int64_t*,
                int64_t*, double*, int64_t*, double*, int64_t*, int64_t*, double*, void*)
{
    return h ? h->fail(KC_EUNSUPPORTED, "mrg not built") : KC_EINVAL;
}
int kcenter_assign(kc_handle* h, const kc_points*, const int64_t*, int64_t, int32_t*, double*,
                   void*)
{
    return h ? h->fail(KC_EUNSUPPORTED, "assign not built") : KC_EINVAL;
}
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
