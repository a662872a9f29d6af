/* Plain C user of the library's ABI: compiles against include/gs.h and links
 * libgs.so.  Uses only the host-side entry points (no device needed) and the
 * argument checks that run before any device work.  Prints one line per
 * check; exits nonzero on the first failure. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "gs.h"

#define CHECK(c, msg)                                  \
    do {                                               \
        if (!(c)) {                                    \
            fprintf(stderr, "FAIL: %s\n", msg);        \
            return 1;                                  \
        }                                              \
        printf("ok: %s\n", msg);                       \
    } while (0)

int main(void) {
    CHECK(gs_version() > 0, "gs_version");
    CHECK(gs_strerror(GS_ERR_INVALID_ARG) != NULL, "gs_strerror");

    /* db2 taps sum to 1 (m0(0) = 1) and have unit energy sum h_k^2 = 1/2 */
    double h[4];
    CHECK(gs_filter_taps(2, h) == GS_OK, "gs_filter_taps(2)");
    double s = 0, e = 0;
    for (int k = 0; k < 4; ++k) {
        s += h[k];
        e += h[k] * h[k];
    }
    CHECK(fabs(s - 1.0) < 1e-14 && fabs(e - 0.5) < 1e-14, "db2 taps: sum 1, energy 1/2");

    /* basis values at xi = 0: the interior scale D(0) = 2^{-J/2} phi-hat(0) = 2^{-J/2} */
    const double xi = 0.0;
    double out[2 * (2 * 2 + 1)];
    CHECK(gs_eval_basis_1d(5, 2, 1, &xi, out) == GS_OK, "gs_eval_basis_1d");
    CHECK(fabs(out[2 * 2] - pow(2.0, -2.5)) < 1e-14 && fabs(out[2 * 2 + 1]) < 1e-14, "D(0) = 2^{-J/2}");

    /* argument checks happen before any device work */
    gs_plan_t* plan = NULL;
    CHECK(gs_plan(&plan, 3, 5, 2, 10, &xi, NULL, GS_F64, NULL) == GS_ERR_INVALID_ARG, "gs_plan rejects dim 3");
    CHECK(gs_plan(&plan, 1, 5, 9, 1, &xi, NULL, GS_F64, NULL) == GS_ERR_UNSUPPORTED, "gs_plan rejects p 9");
    CHECK(gs_apply_T(NULL, &xi, out, 0, NULL) == GS_ERR_INVALID_ARG, "gs_apply_T rejects NULL plan");
    gs_plan_t* plans[2] = {NULL, NULL};
    gs_plan_desc descs[2] = {{1, 5, 9, GS_F64, 1, &xi, NULL}, {1, 5, 2, GS_F64, 1, &xi, NULL}};
    CHECK(gs_plan_batch(plans, 0, descs, NULL) == GS_ERR_INVALID_ARG, "gs_plan_batch rejects count 0");
    CHECK(gs_plan_batch(plans, 2, NULL, NULL) == GS_ERR_INVALID_ARG, "gs_plan_batch rejects NULL descs");
    CHECK(gs_plan_batch(plans, 2, descs, NULL) == GS_ERR_UNSUPPORTED && !plans[0] && !plans[1],
          "gs_plan_batch fails as a whole on an unsupported descriptor");
    gs_cnn_t* cnn = NULL;
    CHECK(gs_cnn_create(&cnn, 0, 8, 1) == GS_ERR_INVALID_ARG, "gs_cnn_create rejects height 0");
    CHECK(gs_cnn_param_count() == 38016, "gs_cnn_param_count");
    gs_destroy(NULL);
    gs_cnn_destroy(NULL);
    printf("all C ABI checks passed\n");
    return 0;
}
