/* A plain C99 consumer of include/sgm.h: compiles the header as C (no C++ or
 * HIP types may leak into it), links libsgm.so and exercises the calls that
 * need no GPU (status strings, argument checks before any device call). */
#include <stdio.h>
#include <string.h>

#include "sgm.h"

static int fails = 0;
#define CHECK(cond)                                             \
    do {                                                        \
        if (!(cond)) {                                          \
            fprintf(stderr, "line %d: %s\n", __LINE__, #cond);  \
            ++fails;                                            \
        }                                                       \
    } while (0)

int main(void) {
    CHECK(strcmp(sgm_status_string(SGM_OK), "ok") == 0);
    CHECK(strcmp(sgm_status_string(SGM_ERR_SINGULAR), "singular system") == 0);
    CHECK(sgm_version() >= 1);

    /* null arguments are rejected before any device call */
    sgm_plan plan = NULL;
    CHECK(sgm_plan_create(NULL, NULL, &plan) == SGM_ERR_INVALID_ARG);
    CHECK(plan == NULL);
    CHECK(strstr(sgm_last_error(), "null") != NULL);
    CHECK(sgm_forward(NULL, NULL, NULL, NULL) == SGM_ERR_INVALID_ARG);
    CHECK(sgm_backward(NULL, NULL, NULL, NULL) == SGM_ERR_INVALID_ARG);
    CHECK(sgm_helmholtz_solve(NULL, 1.0, NULL, NULL, NULL) == SGM_ERR_INVALID_ARG);
    CHECK(sgm_biharmonic_solve(NULL, NULL, NULL, NULL) == SGM_ERR_INVALID_ARG);
    int order[3] = {1, 0, 0};
    CHECK(sgm_project_derivative(NULL, NULL, order, NULL, NULL, NULL) == SGM_ERR_INVALID_ARG);

    /* a descriptor the plan rules reject (Dirichlet needs N >= 3) */
    sgm_plan_desc d;
    memset(&d, 0, sizeof d);
    d.ndim = 2;
    d.basis = SGM_SHEN_DIRICHLET;
    d.N = 2;
    d.M1 = 8;
    d.M2 = 1;
    d.kind_last = SGM_R2C;
    CHECK(sgm_plan_create(&d, NULL, &plan) == SGM_ERR_UNSUPPORTED_SIZE);
    CHECK(plan == NULL);

    if (fails) return 1;
    printf("C ABI consumer: ok\n");
    return 0;
}
