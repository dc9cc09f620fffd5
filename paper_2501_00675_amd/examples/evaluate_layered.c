/*
 * Using the library from C, with no Python: build a small leveled graph, evaluate it for many sample points at
 * FP64 and FP32-rescaled, then submit the same samples to a server and wait for the result.
 *
 * The graph is a complete layered graph, widths 1, 2, 3, 2, 1, whose edges into level l all carry the same
 * factor w_l(x) = a_l / (1 + b_l |x - k_l|^2).  Every root-to-final path then has the same product, and there are
 * d_1 d_2 d_3 d_4 = 1 * 2 * 3 * 2 = 12 of them (d_l = in-degree of level l), so the sum over paths has the closed
 * form V(x) = prod_l d_l w_l(x), which this program checks every result against.
 *
 * Build (the library's build step does this):
 *   gcc -std=c11 -O2 -D__HIP_PLATFORM_AMD__ -I include -I /opt/rocm/include evaluate_layered.c \
 *       -L <dir of libcosdag.so> -lcosdag -L /opt/rocm/lib -lamdhip64 -lm -o evaluate_layered
 * Exit status: 0 when every check passes, 1 on a failed check or call, 77 when no HIP device is present.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "cos.h"

#define L_LEVELS 4
#define N_SAMPLES 3000

static int fail_cos(const char *what, cos_status st) {
    fprintf(stderr, "%s failed (%d): %s\n", what, (int)st, cos_last_error());
    return 1;
}

static int fail_hip(const char *what, hipError_t err) {
    fprintf(stderr, "%s failed: %s\n", what, hipGetErrorString(err));
    return 1;
}

/* uniform in [-1, 1) from a 64-bit linear congruential generator (Knuth's MMIX constants) */
static double uniform(uint64_t *state) {
    *state = *state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

int main(void) {
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev < 1) {
        printf("no HIP device\n");
        return 77;
    }
    const int64_t widths[L_LEVELS + 1] = {1, 2, 3, 2, 1};
    const double a_l[L_LEVELS] = {0.75, -1.25, 0.5, 2.0};
    const double b_l[L_LEVELS] = {1.0, 0.5, 2.0, 0.25};
    const double k_l[L_LEVELS][3] = {{0.1, -0.2, 0.3}, {-0.5, 0.0, 0.25}, {0.0, 0.4, -0.1}, {0.2, 0.2, 0.2}};

    /* every pair of consecutive levels fully connected; node ids are global and level-contiguous */
    int64_t per_level[L_LEVELS], first[L_LEVELS + 1], n_edges = 0;
    first[0] = 0;
    for (int l = 1; l <= L_LEVELS; ++l) {
        first[l] = first[l - 1] + widths[l - 1];
        per_level[l - 1] = widths[l - 1] * widths[l];
        n_edges += per_level[l - 1];
    }
    int32_t *src = malloc(sizeof(int32_t) * n_edges), *dst = malloc(sizeof(int32_t) * n_edges);
    double *a = malloc(sizeof(double) * n_edges), *b = malloc(sizeof(double) * n_edges);
    double *k = malloc(sizeof(double) * 3 * n_edges);
    int64_t e = 0;
    for (int l = 1; l <= L_LEVELS; ++l)
        for (int64_t j = 0; j < widths[l]; ++j)
            for (int64_t i = 0; i < widths[l - 1]; ++i, ++e) {
                src[e] = (int32_t)(first[l - 1] + i);
                dst[e] = (int32_t)(first[l] + j);
                a[e] = a_l[l - 1];
                b[e] = b_l[l - 1];
                for (int c = 0; c < 3; ++c)
                    k[3 * e + c] = k_l[l - 1][c];
            }

    cos_graph *g = NULL;
    cos_status st = cos_create_graph(L_LEVELS, widths, per_level, src, dst, a, b, k, &g);
    free(src), free(dst), free(a), free(b), free(k);
    if (st != COS_OK)
        return fail_cos("cos_create_graph", st);
    cos_graph_info info;
    if ((st = cos_graph_get_info(g, &info)) != COS_OK)
        return fail_cos("cos_graph_get_info", st);
    printf("graph: L=%d, %lld nodes, %lld edges, fused plan bits 0x%x\n", info.L, (long long)info.n_nodes,
           (long long)info.n_edges, (unsigned)info.fused_mask);

    /* samples as rows [3][S] on the host, then on the device */
    static double x[3 * N_SAMPLES], ref[N_SAMPLES], y[N_SAMPLES];
    uint64_t state = 12345;
    for (int i = 0; i < 3 * N_SAMPLES; ++i)
        x[i] = 2.0 * uniform(&state);
    for (int s = 0; s < N_SAMPLES; ++s) {
        ref[s] = 1.0;
        for (int l = 0; l < L_LEVELS; ++l) {
            double r2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double d = x[c * N_SAMPLES + s] - k_l[l][c];
                r2 += d * d;
            }
            const double d_l = (double)widths[l];  /* in-degree of level l+1 in a complete layered graph */
            ref[s] *= d_l * a_l[l] / (1.0 + b_l[l] * r2);
        }
    }
    double *x_dev = NULL, *y_dev = NULL;
    hipError_t err = hipMalloc((void **)&x_dev, sizeof x);
    if (err == hipSuccess)
        err = hipMalloc((void **)&y_dev, sizeof y);
    if (err == hipSuccess)
        err = hipMemcpy(x_dev, x, sizeof x, hipMemcpyHostToDevice);
    if (err != hipSuccess)
        return fail_hip("device buffers", err);

    const cos_precision precs[2] = {COS_FP64, COS_FP32_RESCALED};
    const double tol[2] = {1e-12, 1e-5};
    const char *names[2] = {"FP64", "FP32-rescaled"};
    for (int p = 0; p < 2; ++p) {
        /* NULL workspace: the library allocates it in stream order; stream 0 */
        if ((st = cos_evaluate(g, x_dev, N_SAMPLES, precs[p], y_dev, NULL, NULL, 0, NULL)) != COS_OK)
            return fail_cos("cos_evaluate", st);
        if ((err = hipMemcpy(y, y_dev, sizeof y, hipMemcpyDeviceToHost)) != hipSuccess)
            return fail_hip("hipMemcpy", err);
        double worst = 0.0;
        for (int s = 0; s < N_SAMPLES; ++s)
            worst = fmax(worst, fabs(y[s] - ref[s]) / fabs(ref[s]));
        printf("cos_evaluate %s: max relative error %.3e against the closed form\n", names[p], worst);
        if (!(worst <= tol[p])) {
            fprintf(stderr, "%s: error above %.0e\n", names[p], tol[p]);
            return 1;
        }
    }

    /* the same samples through a server: the result is bit-identical to cos_evaluate's */
    if ((st = cos_evaluate(g, x_dev, N_SAMPLES, COS_FP64, y_dev, NULL, NULL, 0, NULL)) != COS_OK)
        return fail_cos("cos_evaluate", st);
    if ((err = hipMemcpy(y, y_dev, sizeof y, hipMemcpyDeviceToHost)) != hipSuccess)
        return fail_hip("hipMemcpy", err);
    double *z_dev = NULL;
    static double z[N_SAMPLES];
    if ((err = hipMalloc((void **)&z_dev, sizeof z)) != hipSuccess)
        return fail_hip("hipMalloc", err);
    cos_server *srv = NULL;
    int32_t gid = -1;
    uint64_t ticket = 0;
    cos_req_stats rs;
    if ((st = cos_server_create((uint64_t)64 << 20, 4, &srv)) != COS_OK)
        return fail_cos("cos_server_create", st);
    if ((st = cos_server_add_graph(srv, g, &gid)) != COS_OK)
        return fail_cos("cos_server_add_graph", st);
    if ((st = cos_server_submit(srv, gid, x_dev, N_SAMPLES, COS_FP64, z_dev, NULL, &ticket)) != COS_OK)
        return fail_cos("cos_server_submit", st);
    if ((st = cos_server_wait(srv, ticket, &rs)) != COS_OK)
        return fail_cos("cos_server_wait", st);
    if ((err = hipMemcpy(z, z_dev, sizeof z, hipMemcpyDeviceToHost)) != hipSuccess)
        return fail_hip("hipMemcpy", err);
    int same = 1;
    for (int s = 0; s < N_SAMPLES; ++s)
        same &= y[s] == z[s] || (isnan(y[s]) && isnan(z[s]));
    printf("server: request took %d step(s), %s cos_evaluate\n", rs.steps, same ? "bit-identical to" : "DIFFERS from");
    if (!same)
        return 1;

    /* a rejected call: the status says why, cos_last_error gives the message */
    const int64_t bad_widths[2] = {2, 1};
    const int64_t one = 1;
    const int32_t s0 = 0, d0 = 2;
    const double a0 = 1.0, b0 = 0.0, k0[3] = {0, 0, 0};
    cos_graph *bad = NULL;
    st = cos_create_graph(1, bad_widths, &one, &s0, &d0, &a0, &b0, k0, &bad);
    printf("invalid graph refused: status %d (%s)\n", (int)st, cos_last_error());
    if (st != COS_EINVAL || bad != NULL)
        return 1;

    cos_server_destroy(srv);
    cos_destroy_graph(g);
    hipFree(x_dev), hipFree(y_dev), hipFree(z_dev);
    printf("all checks passed\n");
    return 0;
}
