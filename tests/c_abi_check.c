/* Compiled by the ABI tests as plain C99 and linked against libhs.so: the
 * header must be valid C and every declared entry point must resolve. */
#include <stdio.h>

#include "hs.h"

int main(void) {
    const void *fns[] = {
        (const void *)hs_plan_desc_init,       (const void *)hs_plan_create,
        (const void *)hs_plan_create_in,       (const void *)hs_plan_workspace_bytes,
        (const void *)hs_plan_destroy,         (const void *)hs_sum_1d,
        (const void *)hs_sum_batched,          (const void *)hs_sum_2d,
        (const void *)hs_get_norm,             (const void *)hs_quantize_f16,
        (const void *)hs_plan_set_timing,      (const void *)hs_plan_get_timing,
        (const void *)hs_plan_set_graph,       (const void *)hs_plan_graph_info,
        (const void *)hs_plan_set_launch,      (const void *)hs_plan_get_launch,
        (const void *)hs_plan_tune_batched,    (const void *)hs_status_string,
        (const void *)hs_last_error,
    };
    hs_plan_desc d;
    size_t bytes = 0;
    hs_plan_desc_init(&d);
    if (hs_plan_workspace_bytes(&d, &bytes) != HS_OK || bytes == 0) return 1;
    if (hs_plan_create(NULL, NULL) != HS_ERR_ARG) return 2;
    printf("%d entry points, default workspace %zu bytes, H=%d: %s\n", (int)(sizeof fns / sizeof fns[0]), bytes,
           d.harmonics, hs_status_string(HS_OK));
    return 0;
}
