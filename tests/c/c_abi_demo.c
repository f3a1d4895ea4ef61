/*
 * c_abi_demo.c -- the renderer's C ABI used from plain C, checked against the FP64 oracle.
 *
 * TEST PROGRAM.  `c_abi_demo host` exercises the calls that need no GPU (version, argument
 * errors, removal/split tests and the split of Gaussians on host arrays); `c_abi_demo gpu`
 * renders five Gaussians into a 24 x 16 view through device buffers allocated with the HIP
 * runtime, runs the backward pass with the depth cotangent 1/P, and compares both with the
 * oracle library (norm-wise 1e-4 for depth and normals, 1e-5 absolute for alpha, 1e-3
 * norm-wise for the gradients).  Exit status 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fmb.h"

static const double kPi = 3.14159265358979323846;

/* the oracle's C entry points (oracle/fmb_oracle.c) */
void fmbo_pixel_rays(int64_t p, const int32_t *view, const int32_t *row, const int32_t *col,
                     const double *w2c, const double *intr, double *orig, double *dir);
int fmbo_render(int32_t n, const double *means, const double *prec, const double *weights,
                const double *colors, const double *betas, double eta, int64_t p, const double *orig,
                const double *dir, const int32_t *view, const double *w2c_a, const double *intr_a,
                const double *w2c_b, const double *intr_b, double *depth, double *alpha, double *normal,
                double *flow, double *color, int n_threads);
int fmbo_backward(int32_t n, const double *means, const double *prec, const double *weights,
                  const double *colors, const double *betas, double eta, int64_t p, const double *orig,
                  const double *dir, const int32_t *view, const double *w2c_a, const double *intr_a,
                  const double *w2c_b, const double *intr_b, const double *g_depth, const double *g_alpha,
                  const double *g_normal, const double *g_flow, const double *g_color, double *g_means,
                  double *g_prec, double *g_weights, double *g_colors, double *g_betas, int n_threads);

#define CHECK(cond, msg)                                                                           \
    do {                                                                                           \
        if (!(cond)) {                                                                             \
            fprintf(stderr, "FAIL %s (line %d): %s\n", msg, __LINE__, fmb_last_error());           \
            return 1;                                                                              \
        }                                                                                          \
    } while (0)

#define HIP(x) CHECK((x) == hipSuccess, #x)

static double normwise(const float *a, const double *b, int n)
{
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i) {
        num += ((double)a[i] - b[i]) * ((double)a[i] - b[i]);
        den += b[i] * b[i];
    }
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

static int host_checks(void)
{
    CHECK(fmb_abi_version() == FMB_ABI_VERSION, "ABI version");
    CHECK(fmb_render(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == FMB_ERR_INVALID_ARG, "NULL scene");
    CHECK(strlen(fmb_last_error()) > 0, "error message");
    const float w[5] = {1.0f, 1.0f, 1.0f, 1.0f, 0.0f};
    uint8_t rm[5];
    CHECK(fmb_prune_mask(5, w, 1.5f, rm) == FMB_OK, "prune mask");
    CHECK(rm[4] == 1 && rm[0] == 0, "prune mask values");
    /* an axis-aligned Gaussian splits along x into mu +- 0.3 sqrt(2/pi) */
    const float mu[3] = {0.0f, 0.0f, 0.0f}, pr[6] = {1.0f / 0.3f, 0.0f, 0.0f, 1.0f / 0.1f, 0.0f, 1.0f / 0.05f};
    const float lam[1] = {1.0f}, nw[2] = {0.0f, 0.0f};
    float om[6], op[12], ow[2];
    CHECK(fmb_split_gaussians(1, mu, pr, lam, NULL, nw, NULL, om, op, ow, NULL) == FMB_OK, "split");
    const double d = 0.3 * sqrt(2.0 / kPi);
    CHECK(fabs(om[0] - d) < 1e-6 && fabs(om[3] + d) < 1e-6 && fabs(om[1]) < 1e-7, "split means");
    CHECK(fabs(op[0] - 1.0 / (0.3 * sqrt(1.0 - 2.0 / kPi))) < 1e-4 * op[0], "split precision");
    printf("host checks OK\n");
    return 0;
}

static int gpu_checks(void)
{
    enum { N = 5, H = 16, W = 24, P = H * W };
    const float means[N * 3] = {0.0f, 0.0f, 0.0f,  0.3f, 0.1f, 0.2f,  -0.25f, -0.1f, 0.1f,
                                0.1f, 0.3f, -0.2f, -0.1f, -0.3f, 0.3f};
    const float s[N] = {0.2f, 0.15f, 0.1f, 0.12f, 0.18f};
    float prec[N * 6], weights[N], betas[2] = {21.4f, 3.14f};
    for (int i = 0; i < N; ++i) {
        const float u[6] = {1.0f / s[i], 0.0f, 0.0f, 1.0f / s[i], 0.0f, 1.0f / s[i]};
        memcpy(prec + 6 * i, u, sizeof u);
        weights[i] = 0.5f + 0.1f * (float)i;
    }
    /* camera at (0, 0, -3) looking along +z: x_cam = x_world + (0, 0, 3) */
    const float w2c[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3};
    const float intr[4] = {(float)H, (float)H, W / 2.0f, H / 2.0f};
    const int32_t hw[2] = {H, W};

    float *d_means, *d_prec, *d_weights, *d_betas, *d_w2c, *d_intr;
    float *d_depth, *d_alpha, *d_normal, *d_stash, *d_gd, *d_gm, *d_gp, *d_gw, *d_gb;
    HIP(hipMalloc((void **)&d_means, sizeof means));
    HIP(hipMalloc((void **)&d_prec, sizeof prec));
    HIP(hipMalloc((void **)&d_weights, sizeof weights));
    HIP(hipMalloc((void **)&d_betas, sizeof betas));
    HIP(hipMalloc((void **)&d_w2c, sizeof w2c));
    HIP(hipMalloc((void **)&d_intr, sizeof intr));
    HIP(hipMalloc((void **)&d_depth, P * sizeof(float)));
    HIP(hipMalloc((void **)&d_alpha, P * sizeof(float)));
    HIP(hipMalloc((void **)&d_normal, 3 * P * sizeof(float)));
    HIP(hipMalloc((void **)&d_stash, 8 * P * sizeof(float)));
    HIP(hipMalloc((void **)&d_gd, P * sizeof(float)));
    HIP(hipMalloc((void **)&d_gm, 3 * N * sizeof(float)));
    HIP(hipMalloc((void **)&d_gp, 6 * N * sizeof(float)));
    HIP(hipMalloc((void **)&d_gw, N * sizeof(float)));
    HIP(hipMalloc((void **)&d_gb, 2 * sizeof(float)));
    HIP(hipMemcpy(d_means, means, sizeof means, hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_prec, prec, sizeof prec, hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_weights, weights, sizeof weights, hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_betas, betas, sizeof betas, hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_w2c, w2c, sizeof w2c, hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_intr, intr, sizeof intr, hipMemcpyHostToDevice));
    float gd[P];
    for (int r = 0; r < P; ++r) gd[r] = 1.0f / P;
    HIP(hipMemcpy(d_gd, gd, sizeof gd, hipMemcpyHostToDevice));

    fmb_scene *scene = NULL;
    CHECK(fmb_scene_create(&scene, N, d_means, d_prec, d_weights, d_betas, 1.0f) == FMB_OK, "scene create");
    CHECK(fmb_set_cameras(scene, 1, d_w2c, d_intr, hw, NULL, NULL) == FMB_OK, "set cameras");
    CHECK(fmb_num_rays(scene) == P, "ray count");
    CHECK(fmb_render(scene, d_depth, d_alpha, d_normal, NULL, NULL, d_stash, NULL) == FMB_OK, "render");
    CHECK(fmb_backward(scene, d_gd, NULL, NULL, NULL, NULL, d_depth, NULL, d_stash, d_gm, d_gp, d_gw, NULL,
                       d_gb, NULL) == FMB_OK, "backward");
    HIP(hipDeviceSynchronize());
    float depth[P], alpha[P], normal[3 * P], gm[3 * N], gp[6 * N], gw[N], gb[2];
    HIP(hipMemcpy(depth, d_depth, sizeof depth, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(alpha, d_alpha, sizeof alpha, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(normal, d_normal, sizeof normal, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(gm, d_gm, sizeof gm, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(gp, d_gp, sizeof gp, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(gw, d_gw, sizeof gw, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(gb, d_gb, sizeof gb, hipMemcpyDeviceToHost));
    CHECK(fmb_scene_destroy(scene) == FMB_OK, "destroy");

    /* oracle on the same float inputs, in double */
    double dm[3 * N], dp[6 * N], dw[N], db[2] = {betas[0], betas[1]}, de[12], dk[4];
    for (int i = 0; i < 3 * N; ++i) dm[i] = means[i];
    for (int i = 0; i < 6 * N; ++i) dp[i] = prec[i];
    for (int i = 0; i < N; ++i) dw[i] = weights[i];
    for (int i = 0; i < 12; ++i) de[i] = w2c[i];
    for (int i = 0; i < 4; ++i) dk[i] = intr[i];
    int32_t view[P], row[P], col[P];
    double orig[3 * P], dir[3 * P], rd[P], ra[P], rn[3 * P], rgd[P];
    for (int r = 0; r < P; ++r) {
        view[r] = 0;
        row[r] = r / W;
        col[r] = r % W;
        rgd[r] = gd[r];
    }
    fmbo_pixel_rays(P, view, row, col, de, dk, orig, dir);
    CHECK(fmbo_render(N, dm, dp, dw, NULL, db, 1.0, P, orig, dir, view, de, dk, NULL, NULL, rd, ra, rn, NULL,
                      NULL, 1) == 0, "oracle render");
    double rgm[3 * N], rgp[6 * N], rgw[N], rgb[2];
    CHECK(fmbo_backward(N, dm, dp, dw, NULL, db, 1.0, P, orig, dir, view, de, dk, NULL, NULL, rgd, NULL, NULL,
                        NULL, NULL, rgm, rgp, rgw, NULL, rgb, 1) == 0, "oracle backward");
    double amax = 0.0;
    for (int r = 0; r < P; ++r) amax = fmax(amax, fabs((double)alpha[r] - ra[r]));
    const double ed = normwise(depth, rd, P), en = normwise(normal, rn, 3 * P);
    const double egm = normwise(gm, rgm, 3 * N), egp = normwise(gp, rgp, 6 * N), egw = normwise(gw, rgw, N);
    const double egb = normwise(gb, rgb, 2);
    printf("depth %.3e alpha %.3e normal %.3e | grad means %.3e prec %.3e weights %.3e betas %.3e\n", ed, amax, en,
           egm, egp, egw, egb);
    CHECK(ed <= 1e-4 && en <= 1e-4 && amax <= 1e-5, "forward parity");
    CHECK(egm <= 1e-3 && egp <= 1e-3 && egw <= 1e-3 && egb <= 1e-3, "gradient parity");
    printf("gpu checks OK\n");
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 2) {
        fprintf(stderr, "usage: %s host|gpu\n", argv[0]);
        return 2;
    }
    if (strcmp(argv[1], "host") == 0) return host_checks();
    if (strcmp(argv[1], "gpu") == 0) return host_checks() || gpu_checks();
    return 2;
}
