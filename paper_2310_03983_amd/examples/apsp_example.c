/*
 * apsp_example.c -- drives libapsp through its C ABI only (no Python, no
 * torch): builds a small directed graph, solves it with blocked
 * Floyd-Warshall and R-Kleene, recovers one shortest path from the
 * predecessor matrix and prints it.  Given a cost-model file (the text
 * format of apsp_costmodel_load, e.g. data/costmodel_mlp.txt), it also
 * loads the model and prints the plan it picks for a large sparse graph.
 *
 *   cc -I include paper_2310_03983_amd/examples/apsp_example.c \
 *      -L paper_2310_03983_amd -lapsp -L /opt/rocm/lib -lamdhip64 \
 *      -Wl,-rpath,paper_2310_03983_amd -Wl,-rpath,/opt/rocm/lib -o apsp_example
 *   ./apsp_example [model.txt]    (needs a GPU; exit status 0 on success)
 *
 * Device memory comes straight from the HIP runtime (hipMalloc/hipMemcpy are
 * declared below so that the example needs no HIP headers).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "apsp.h"

typedef int hipError_t;
extern hipError_t hipMalloc(void **ptr, size_t size);
extern hipError_t hipFree(void *ptr);
extern hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, int kind);
extern hipError_t hipDeviceSynchronize(void);
#define H2D 1
#define D2H 2

#define N 6
#define INF APSP_INF_I32

static int check(apsp_status_t st, const char *what)
{
    if (st != APSP_OK) {
        fprintf(stderr, "%s failed (%d): %s\n", what, (int)st, apsp_last_error());
        return 1;
    }
    return 0;
}

int main(int argc, char **argv)
{
    /* 0 -> 1 -> 2 -> 3 -> 4 -> 5 chain of cost 1 plus a costly shortcut 0 -> 5 */
    int32_t W[N * N];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) W[i * N + j] = (i == j) ? 0 : INF;
    for (int i = 0; i + 1 < N; ++i) W[i * N + i + 1] = 1;
    W[0 * N + 5] = 10;

    apsp_ctx_t *ctx = NULL;
    if (check(apsp_create(&ctx, 0), "apsp_create")) return 1;
    printf("%s\n", apsp_version());

    int32_t *dW = NULL, *dD = NULL, *dP = NULL;
    if (hipMalloc((void **)&dW, sizeof W) || hipMalloc((void **)&dD, sizeof W) ||
        hipMalloc((void **)&dP, sizeof W)) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    hipMemcpy(dW, W, sizeof W, H2D);
    int64_t bad = -1;
    if (check(apsp_validate(ctx, APSP_I32, N, dW, N, NULL, &bad), "apsp_validate")) return 1;

    int32_t D[N * N], D2[N * N], P[N * N];
    hipMemcpy(dD, W, sizeof W, H2D);
    if (check(apsp_fw(ctx, APSP_I32, N, dD, N, NULL, NULL), "apsp_fw")) return 1;
    hipMemcpy(D, dD, sizeof D, D2H);
    hipMemcpy(dD, W, sizeof W, H2D);
    if (check(apsp_rkleene(ctx, APSP_I32, N, dD, N, NULL, NULL), "apsp_rkleene")) return 1;
    if (check(apsp_predecessors(ctx, APSP_I32, N, dD, N, dW, N, dP, N, NULL), "apsp_predecessors")) return 1;
    hipMemcpy(D2, dD, sizeof D2, D2H);
    hipMemcpy(P, dP, sizeof P, D2H);
    hipDeviceSynchronize();

    int ok = 1;
    for (int e = 0; e < N * N; ++e) ok &= (D[e] == D2[e]);
    ok &= (D[0 * N + 5] == 5);               /* the chain beats the shortcut */
    int path[N + 1], len = 0, v = 5;
    while (v != 0 && len <= N) { path[len++] = v; v = P[0 * N + v]; if (v < 0) break; }
    path[len++] = 0;
    printf("dist(0,5) = %d, path:", D[5]);
    for (int t = len - 1; t >= 0; --t) printf(" %d", path[t]);
    printf("\n");
    ok &= (len == N);

    if (argc > 1) {
        /* the trained cost model picks the plan apsp_solve would run */
        apsp_opts_t plan;
        int32_t choice = -1;
        if (check(apsp_costmodel_load(ctx, argv[1]), "apsp_costmodel_load")) return 1;
        if (check(apsp_plan(ctx, APSP_I32, 16384, 0.01, 1, 1, &plan, &choice), "apsp_plan")) return 1;
        printf("plan for n=16384, density 0.01: candidate %d (algo %d, block %d, cutover %d, flags %d)\n",
               (int)choice, (int)plan.algo, (int)plan.block, (int)plan.cutover, (int)plan.flags);
        ok &= (choice >= 0);
    }

    hipFree(dW); hipFree(dD); hipFree(dP);
    apsp_destroy(ctx);
    printf(ok ? "example ok\n" : "example FAILED\n");
    return ok ? 0 : 1;
}
