/* The 2-D transverse-magnetic C-ABI used from plain C (no Python, no torch):
 * the PEC cavity (0,1)^2 with the constant current j = 1 (Section 6), on a
 * 3 x 3 Cartesian mesh of four triangles per cell that meet at the cell's
 * centre, P2 fields in FP64, CMCG to 1e-10 and the filtered fields, once
 * through the host-pointer calls and once through the device-pointer calls
 * (hipMalloc'd current and outputs on a stream of our own); both must agree
 * bit for bit.  Writes mesh, current and fields to argv[1] for comparison
 * with the FP64 oracle.
 *
 * Exit status: 0 on success, 1 on a library error or a mismatch. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cmcg.h"

#define N 3          /* cells per side */
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
    /* corners (i, j) first, then the cell centres; cell c = ci + N cj holds
     * triangles 4c + s (s = bottom, right, top, left side), each listed as
     * (centre, side start, side end) counter-clockwise, so that local edge 0
     * (opposite the centre) is the cell side */
    const int64_t ncorner = (int64_t)(N + 1) * (N + 1), nv = ncorner + (int64_t)N * N, K = 4LL * N * N;
    double* xy = malloc(sizeof(double) * 2 * nv);
    int64_t* tri = malloc(sizeof(int64_t) * 3 * K);
    int8_t* tag = calloc((size_t)K * 3, 1);
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
            xy[2 * (i + (N + 1) * j)] = (double)i / N;
            xy[2 * (i + (N + 1) * j) + 1] = (double)j / N;
        }
    for (int cj = 0; cj < N; ++cj)
        for (int ci = 0; ci < N; ++ci) {
            const int64_t c = ci + (int64_t)N * cj, centre = ncorner + c;
            xy[2 * centre] = (ci + 0.5) / N;
            xy[2 * centre + 1] = (cj + 0.5) / N;
            const int64_t corner[4] = {ci + (N + 1) * cj, ci + 1 + (N + 1) * cj, ci + 1 + (N + 1) * (cj + 1),
                                       ci + (N + 1) * (cj + 1)};
            const int on_wall[4] = {cj == 0, ci == N - 1, cj == N - 1, ci == 0};
            for (int s = 0; s < 4; ++s) {
                const int64_t t = 4 * c + s;
                tri[3 * t] = centre;
                tri[3 * t + 1] = corner[s];
                tri[3 * t + 2] = corner[(s + 1) % 4];
                if (on_wall[s]) tag[3 * t] = CMCG_TAG_PEC;
            }
        }
    cmcg_mesh* m = NULL;
    cmcg_space* sp = NULL;
    check(cmcg_mesh2d_create(nv, xy, K, tri, tag, &m), "mesh2d");
    int dim = 0;
    check(cmcg_mesh_dim(m, &dim), "mesh_dim");
    check(cmcg_space_create(m, Q, CMCG_FP64, &sp), "space");
    int q, Np, Nfp;
    int64_t K2, ndof;
    check(cmcg_space_info(sp, &q, &Np, &Nfp, &K2, &ndof), "space_info");

    /* eps 1 or 2 by triangle parity, mu = 1, j = 1 at every node */
    double* eps = malloc(sizeof(double) * K);
    double* mu = malloc(sizeof(double) * K);
    double* j = malloc(sizeof(double) * K * Np);
    for (int64_t t = 0; t < K; ++t) {
        eps[t] = (t % 2) ? 2.0 : 1.0;
        mu[t] = 1.0;
    }
    for (int64_t i = 0; i < K * Np; ++i) j[i] = 1.0;
    cmcg_options o;
    cmcg_options_default(&o);
    o.tol = 1e-10;
    o.max_iter = 500;

    /* 1: host pointers, default stream */
    cmcg_problem* ph = NULL;
    cmcg_result* rh = NULL;
    check(cmcg_problem_create(sp, eps, mu, NULL, OMEGA, j, NULL, NULL, NULL, &ph), "problem");
    const int st_h = check(cmcg_solve(ph, &o, NULL, NULL, &rh), "solve");
    const size_t ne = (size_t)K * Np, nh = 2 * ne;
    double* fh = malloc(sizeof(double) * (2 * ne + 2 * nh));
    check(cmcg_result_fields(rh, fh, fh + ne, fh + 2 * ne, fh + 2 * ne + nh), "fields");
    cmcg_stats stats;
    check(cmcg_result_stats(rh, &stats), "stats");

    /* 2: device pointers on a stream of our own */
    hipStream_t stream;
    hip_check(hipStreamCreate(&stream), "stream");
    double *jd = NULL, *fre = NULL, *fim = NULL;
    hip_check(hipMalloc((void**)&jd, sizeof(double) * ne), "malloc j");
    hip_check(hipMalloc((void**)&fre, sizeof(double) * ndof), "malloc f");
    hip_check(hipMalloc((void**)&fim, sizeof(double) * ndof), "malloc f");
    hip_check(hipMemcpy(jd, j, sizeof(double) * ne, hipMemcpyHostToDevice), "copy j");
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

    printf("dim=%d K=%lld Np=%d ndof=%lld iters=%d rel_res=%.3e status=%d host/device paths %s\n", dim,
           (long long)K, Np, (long long)ndof, stats.iters, stats.rel_res, st_h, same ? "identical" : "DIFFER");

    FILE* f = fopen(argv[1], "wb");
    if (!f) {
        perror("output");
        return 1;
    }
    const int64_t hdr[3] = {nv, K, Np};
    fwrite(hdr, sizeof(int64_t), 3, f);
    fwrite(xy, sizeof(double), 2 * nv, f);
    fwrite(tri, sizeof(int64_t), 3 * K, f);
    fwrite(tag, 1, 3 * K, f);
    fwrite(eps, sizeof(double), K, f);
    fwrite(fh, sizeof(double), 2 * ne + 2 * nh, f);
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
    free(xy); free(tri); free(tag); free(eps); free(mu); free(j); free(fh); free(fd); free(fd2);
    return (same && dim == 2 && ndof == 3 * K * Np && st_h == CMCG_OK && stats.rel_res <= 1e-10) ? 0 : 1;
}
