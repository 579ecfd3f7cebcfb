/* The C-ABI used from plain C (no Python, no torch): a 48-tetrahedron cube,
 * P2 nodal fields in FP64, a Gaussian current, CMCG to 1e-10 and the
 * filtered fields, once through the host-pointer calls and once through the
 * device-pointer calls (hipMalloc'd inputs and outputs on a stream of our
 * own); both must agree bit for bit.  Writes mesh, inputs and fields to
 * argv[1] for comparison with the FP64 oracle.
 *
 * Exit status: 0 on success, 1 on a library error or a mismatch. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cmcg.h"

#define N 2          /* cubes per axis */
#define Q 2          /* polynomial order */
#define OMEGA (2.0 * 3.14159265358979323846)

static int check(int rc, const char* what) {
    if (rc < 0) {
        fprintf(stderr, "%s: error %d: %s\n", what, rc, cmcg_last_error());
        exit(1);
    }
    return rc;
}

static void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        exit(1);
    }
}

int main(int argc, char** argv) {
    if (argc < 2) {
        fprintf(stderr, "usage: %s OUTPUT\n", argv[0]);
        return 1;
    }
    /* Kuhn split: every cube into six tetrahedra along its main diagonal */
    const int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1), K = 6LL * N * N * N;
    double* xyz = malloc(sizeof(double) * 3 * nv);
    int64_t* tet = malloc(sizeof(int64_t) * 4 * K);
    for (int k = 0; k <= N; ++k)
        for (int j = 0; j <= N; ++j)
            for (int i = 0; i <= N; ++i) {
                const int64_t v = i + (N + 1) * (j + (N + 1) * (int64_t)k);
                xyz[3 * v] = (double)i / N;
                xyz[3 * v + 1] = (double)j / N;
                xyz[3 * v + 2] = (double)k / N;
            }
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t e = 0;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i)
                for (int p = 0; p < 6; ++p, ++e) {
                    int c[3] = {i, j, k};
                    for (int s = 0; s < 4; ++s) {
                        if (s > 0) c[perms[p][s - 1]] += 1;
                        tet[4 * e + s] = c[0] + (N + 1) * (c[1] + (N + 1) * (int64_t)c[2]);
                    }
                }
    cmcg_mesh* m = NULL;
    cmcg_space* sp = NULL;
    check(cmcg_mesh_create(nv, xyz, K, tet, NULL, &m), "mesh");
    check(cmcg_space_create(m, Q, CMCG_FP64, &sp), "space");
    int q, Np, Nfp;
    int64_t K2, ndof;
    check(cmcg_space_info(sp, &q, &Np, &Nfp, &K2, &ndof), "space_info");

    /* inputs: eps 1 or 2 by element parity, e_z Gaussian current at the nodes */
    double* eps = malloc(sizeof(double) * K);
    double* mu = malloc(sizeof(double) * K);
    double* nodes = malloc(sizeof(double) * K * Np * 3);
    double* j = calloc((size_t)K * Np * 3, sizeof(double));
    check(cmcg_space_nodes(sp, nodes), "nodes");
    for (int64_t t = 0; t < K; ++t) {
        eps[t] = (t % 2) ? 2.0 : 1.0;
        mu[t] = 1.0;
    }
    for (int64_t i = 0; i < K * Np; ++i) {
        const double dx = nodes[3 * i] - 0.5, dy = nodes[3 * i + 1] - 0.5, dz = nodes[3 * i + 2] - 0.5;
        j[3 * i + 2] = exp(-(dx * dx + dy * dy + dz * dz) / 0.09);
    }
    cmcg_options o;
    cmcg_options_default(&o);
    o.tol = 1e-10;
    o.max_iter = 500;

    /* 1: host pointers, default stream */
    cmcg_problem* ph = NULL;
    cmcg_result* rh = NULL;
    check(cmcg_problem_create(sp, eps, mu, NULL, OMEGA, j, NULL, NULL, NULL, &ph), "problem");
    const int st_h = check(cmcg_solve(ph, &o, NULL, NULL, &rh), "solve");
    const size_t nf = (size_t)K * Np * 3;
    double* fh = malloc(sizeof(double) * 4 * nf);
    check(cmcg_result_fields(rh, fh, fh + nf, fh + 2 * nf, fh + 3 * nf), "fields");
    cmcg_stats stats;
    check(cmcg_result_stats(rh, &stats), "stats");

    /* 2: device pointers on a stream of our own */
    hipStream_t stream;
    hip_check(hipStreamCreate(&stream), "stream");
    double *jd = NULL, *fre = NULL, *fim = NULL;
    hip_check(hipMalloc((void**)&jd, sizeof(double) * nf), "malloc j");
    hip_check(hipMalloc((void**)&fre, sizeof(double) * ndof), "malloc f");
    hip_check(hipMalloc((void**)&fim, sizeof(double) * ndof), "malloc f");
    hip_check(hipMemcpy(jd, j, sizeof(double) * nf, hipMemcpyHostToDevice), "copy j");
    cmcg_problem* pd = NULL;
    cmcg_result* rd = NULL;
    check(cmcg_problem_create_device(sp, eps, mu, NULL, OMEGA, jd, NULL, NULL, NULL, stream, &pd), "problem_device");
    check(cmcg_solve(pd, &o, NULL, stream, &rd), "solve_device");
    check(cmcg_result_filtered_device(rd, fre, fim, stream), "filtered_device");
    hip_check(hipStreamSynchronize(stream), "sync");
    double* fd = malloc(sizeof(double) * 2 * ndof);
    hip_check(hipMemcpy(fd, fre, sizeof(double) * ndof, hipMemcpyDeviceToHost), "copy f");
    hip_check(hipMemcpy(fd + ndof, fim, sizeof(double) * ndof, hipMemcpyDeviceToHost), "copy f");
    double* fd2 = malloc(sizeof(double) * 2 * ndof);
    check(cmcg_result_filtered_device(rh, fre, fim, NULL), "filtered_device host result");
    hip_check(hipDeviceSynchronize(), "sync");
    hip_check(hipMemcpy(fd2, fre, sizeof(double) * ndof, hipMemcpyDeviceToHost), "copy f");
    hip_check(hipMemcpy(fd2 + ndof, fim, sizeof(double) * ndof, hipMemcpyDeviceToHost), "copy f");
    const int same = memcmp(fd, fd2, sizeof(double) * 2 * ndof) == 0;

    printf("K=%lld Np=%d iters=%d rel_res=%.3e status=%d host/device paths %s\n", (long long)K, Np, stats.iters,
           stats.rel_res, st_h, same ? "identical" : "DIFFER");

    FILE* f = fopen(argv[1], "wb");
    if (!f) {
        perror("output");
        return 1;
    }
    const int64_t hdr[3] = {nv, K, Np};
    fwrite(hdr, sizeof(int64_t), 3, f);
    fwrite(xyz, sizeof(double), 3 * nv, f);
    fwrite(tet, sizeof(int64_t), 4 * K, f);
    fwrite(eps, sizeof(double), K, f);
    fwrite(j, sizeof(double), nf, f);
    fwrite(fh, sizeof(double), 4 * nf, f);
    fclose(f);

    cmcg_result_destroy(rh);
    cmcg_result_destroy(rd);
    cmcg_problem_destroy(ph);
    cmcg_problem_destroy(pd);
    cmcg_space_destroy(sp);
    cmcg_mesh_destroy(m);
    (void)hipFree(jd);
    (void)hipFree(fre);
    (void)hipFree(fim);
    (void)hipStreamDestroy(stream);
    free(xyz); free(tet); free(eps); free(mu); free(nodes); free(j); free(fh); free(fd); free(fd2);
    return (same && st_h == CMCG_OK && stats.rel_res <= 1e-10) ? 0 : 1;
}
