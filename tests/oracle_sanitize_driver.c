/* Runs the C oracle (oracle/gs_oracle.c, linked in) on one scene and camera
 * read from a binary file, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any out-of-bounds access, use after free,
 * leak or undefined operation in the oracle aborts the run.
 *
 * File: int64 n, int32 deg, int32 W, int32 H, int32 0, then FP32 means
 * [n][3], scales [n][3], quats [n][4], opacity [n], sh [n][(deg+1)^2][3],
 * pose [12], intrinsics [4]. Prints the counters and an RGB checksum. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void gso_project_all(const float *means, const float *scales, const float *quats,
                     const float *opacity, const float *sh, int64_t n, int deg, const float pose[12],
                     const float intr[4], int W, int H, double near, double *out);
int gso_render(const float *means, const float *scales, const float *quats, const float *opacity,
               const float *sh, int64_t n, int deg, const float pose[12], const float intr[4],
               int W, int H, double near, const double bg[3], const double margins[4],
               double *rgb, double *depth, double *alpha, double *tfinal, int64_t *counters,
               int64_t var_cap, int32_t *var_pix, double *var_vals, int64_t *n_var,
               int nthreads);
int gso_pixel_trace(const float *means, const float *scales, const float *quats,
                    const float *opacity, const float *sh, int64_t n, int deg, const float pose[12],
                    const float intr[4], int W, int H, double near, double eps_alpha, int i, int j,
                    int cap, double *out);

static float *read_f32(FILE *f, size_t count)
{
    float *p = (float *)malloc(sizeof(float) * (count ? count : 1));
    if (!p || fread(p, sizeof(float), count, f) != count) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n;
    int32_t hdr[4];
    if (fread(&n, sizeof n, 1, f) != 1 || fread(hdr, sizeof(int32_t), 4, f) != 4) return 2;
    const int deg = hdr[0], W = hdr[1], H = hdr[2];
    const size_t nc = (size_t)(deg + 1) * (deg + 1);
    float *means = read_f32(f, (size_t)n * 3), *scales = read_f32(f, (size_t)n * 3);
    float *quats = read_f32(f, (size_t)n * 4), *opacity = read_f32(f, (size_t)n);
    float *sh = read_f32(f, (size_t)n * nc * 3), *pose = read_f32(f, 12), *intr = read_f32(f, 4);
    fclose(f);
    const size_t px = (size_t)W * H;
    double *rgb = malloc(sizeof(double) * px * 3), *depth = malloc(sizeof(double) * px);
    double *alpha = malloc(sizeof(double) * px), *tfin = malloc(sizeof(double) * px);
    double *proj = malloc(sizeof(double) * (size_t)n * 20);
    const int64_t cap = 64;  /* small on purpose: the count past it is still reported */
    int32_t *vp = malloc(sizeof(int32_t) * cap);
    double *vv = malloc(sizeof(double) * cap * 5);
    int64_t cnt[8], nv = 0;
    const double bg[3] = {0.1, 0.2, 0.3}, margins[4] = {2e-3, 2e-3, 2e-5, 1e-5};
    double trace[6 * 32];
    gso_project_all(means, scales, quats, opacity, sh, n, deg, pose, intr, W, H, 0.2, proj);
    const int rc = gso_render(means, scales, quats, opacity, sh, n, deg, pose, intr, W, H, 0.2,
                              bg, margins, rgb, depth, alpha, tfin, cnt, cap, vp, vv, &nv, 2);
    for (int j = 0; j < H; j += 7)
        for (int i = 0; i < W; i += 5)
            gso_pixel_trace(means, scales, quats, opacity, sh, n, deg, pose, intr, W, H, 0.2, 2e-3,
                            i, j, 32, trace);
    double sum = 0.0;
    for (size_t k = 0; k < px * 3; ++k) sum += rgb[k];
    printf("rc %d visible %lld pairs %lld flagged %lld variants %lld checksum %.9f\n", rc,
           (long long)cnt[1], (long long)cnt[3], (long long)cnt[4], (long long)nv, sum);
    free(means); free(scales); free(quats); free(opacity); free(sh); free(pose); free(intr);
    free(rgb); free(depth); free(alpha); free(tfin); free(proj); free(vp); free(vv);
    return rc;
}
