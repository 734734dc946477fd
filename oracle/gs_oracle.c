/*
 * FP64 reference rasteriser for 3D Gaussian splats -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. The GPU renderer shares no code with it.
 *
 * What it computes (the plain definition, no tiling, no sorting network):
 * the paper renders RGB with 3D Gaussian splatting and obtains depth as a
 * by-product of the same rasterisation (Sec. 3.2 "3D Gaussian Splatting as a
 * Drop-in Renderer", Fig. "Rendering RGB and Depth"; the splat model itself is
 * the cited 3DGS of Kerbl et al., Sec. 2.3). Per camera and per pixel centre
 * p = (i + 1/2, j + 1/2):
 *
 *   1. world -> camera with the inverse of the camera-to-world pose;
 *      Gaussians with camera depth z <= near are dropped;
 *   2. 3D covariance  Sigma = R(q) S S^T R(q)^T  (S = diag(scale));
 *   3. EWA projection Sigma' = J W Sigma W^T J^T + 0.3 I, with J the Jacobian
 *      of the pinhole projection at the (field-of-view clamped) mean;
 *   4. colour = max(0, sum_lm k_lm Y_lm(d) + 0.5), d the unit direction from
 *      the camera centre to the mean, Y_lm real SH with Condon-Shortley phase;
 *   5. alpha_g(p) = min(0.99, o_g exp(-1/2 delta^T Sigma'^-1 delta)),
 *      delta = p - (u, v); the candidates of p are the Gaussians with
 *      alpha >= 1/255, ordered by (z, index);
 *   6. front-to-back walk from T = 1: T' = T (1 - alpha); stop (without
 *      the current Gaussian) when T' < 1e-4; otherwise accumulate
 *      alpha T (rgb, z, 1) and set T = T';
 *   7. RGB = acc_rgb + T bg; expected depth = acc_z / acc_w (0 if acc_w = 0);
 *      alpha = acc_w.
 *
 * Every constant is used at its FP32 value (0.99f, 1/255.f, 1e-4f, 0.3f,
 * 1.3f, near as given in FP32) so that FP32 and FP64 take the same decision
 * wherever the margin exceeds rounding.
 *
 * Several results are correct where a decision sits at its threshold within
 * rounding (skip at 1/255, stop at 1e-4, the near plane, contributors at
 * nearly the same depth). For such pixels the oracle additionally enumerates
 * every combination of those decisions and every order of each run of up to
 * four near-tied contributors (bounded; beyond the bound the pixel is counted
 * as unresolved) and reports the alternative results, so a comparator can
 * accept a GPU value matching any of them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ALPHA_MAX ((double)0.99f)
#define ALPHA_MIN ((double)(1.0f / 255.0f))
#define T_MIN ((double)1e-4f)
#define LOWPASS ((double)0.3f)
#define TAN_CLAMP ((double)1.3f)

/* ------------------------------------------------------------- rotation -- */

/* Rotation matrix (row-major) of the unit quaternion q/|q|, q = (w,x,y,z). */
void gso_quat_to_rot(const double q_in[4], double R[9])
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] +
                    q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------- spherical harmonics -- */

/* Associated Legendre function P_l^m(x), m >= 0, including the
 * Condon-Shortley phase (-1)^m, by the standard three-term recurrence. */
static double assoc_legendre(int l, int m, double x)
{
    double pmm = 1.0;
    if (m > 0) {
        double s = sqrt(fmax(0.0, (1.0 - x) * (1.0 + x)));
        double fact = 1.0;
        for (int i = 1; i <= m; ++i) {
            pmm *= -fact * s;
            fact += 2.0;
        }
    }
    if (l == m) return pmm;
    double pmmp1 = x * (2 * m + 1) * pmm;
    if (l == m + 1) return pmmp1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m);
        pmm = pmmp1;
        pmmp1 = pll;
    }
    return pll;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* Real spherical harmonic Y_lm at the unit direction d:
 *   m > 0: sqrt2 K_l^m P_l^m(cos th) cos(m phi)
 *   m = 0:       K_l^0 P_l^0(cos th)
 *   m < 0: sqrt2 K_l^|m| P_l^|m|(cos th) sin(|m| phi)
 * with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). */
double gso_sh_basis(int l, int m, const double d[3])
{
    double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double x = d[0] / nrm, y = d[1] / nrm, z = d[2] / nrm;
    double phi = atan2(y, x);
    int am = m < 0 ? -m : m;
    double K = sqrt((2 * l + 1) / (4 * M_PI) * factorial(l - am) / factorial(l + am));
    double P = assoc_legendre(l, am, z);
    if (m == 0) return K * P;
    if (m > 0) return sqrt(2.0) * K * P * cos(am * phi);
    return sqrt(2.0) * K * P * sin(am * phi);
}

/* colour = max(0, sum_{l<=deg} sum_m coef[l^2+l+m][c] Y_lm(d) + 0.5) */
void gso_sh_color(int deg, const double d[3], const double *coef, double rgb[3])
{
    double acc[3] = {0, 0, 0};
    for (int l = 0; l <= deg; ++l)
        for (int m = -l; m <= l; ++m) {
            double y = gso_sh_basis(l, m, d);
            int k = l * l + l + m;
            for (int c = 0; c < 3; ++c) acc[c] += coef[k * 3 + c] * y;
        }
    for (int c = 0; c < 3; ++c) rgb[c] = fmax(0.0, acc[c] + 0.5);
}

/* ------------------------------------------------------------ projection -- */

typedef struct {
    double R_wc[9], t_wc[3], C[3];
    double fx, fy, cx, cy;
    int W, H;
} camera_t;

static void camera_setup(const float pose[12], const float intr[4], int W, int H,
                         camera_t *cam)
{
    /* pose = [R_cw | C] row-major; R_wc = R_cw^T, t_wc = -R_cw^T C */
    for (int r = 0; r < 3; ++r) {
        cam->C[r] = pose[r * 4 + 3];
        for (int c = 0; c < 3; ++c) cam->R_wc[c * 3 + r] = pose[r * 4 + c];
    }
    for (int r = 0; r < 3; ++r) {
        double s = 0;
        for (int c = 0; c < 3; ++c) s += cam->R_wc[r * 3 + c] * cam->C[c];
        cam->t_wc[r] = -s;
    }
    cam->fx = intr[0]; cam->fy = intr[1]; cam->cx = intr[2]; cam->cy = intr[3];
    cam->W = W; cam->H = H;
}

/* Per-Gaussian projected record (FP64). */
typedef struct {
    double u, v, z;
    double cov[3];    /* Sigma' = [[a, b], [b, c]] incl. low-pass */
    double conic[3];  /* Sigma'^-1 = [[A, B], [B, C]] */
    double o;
    double rgb[3];
    int x0, x1, y0, y1;   /* pixel-centre box of alpha >= ALPHA_MIN (inclusive) */
    int in_front;         /* z > near */
    int near_marginal;    /* |z - near| within the near margin */
    int hits_image;       /* the exact box contains a pixel centre */
} proj_t;

/* Steps 1-4 of the header for one Gaussian. Returns 0 if z is behind
 * (near - margin), 1 otherwise (record filled). */
static int project_one(const camera_t *cam, const float *mean, const float *scale,
                       const float *quat, float opacity, const float *sh, int deg,
                       double near, double eps_near, proj_t *P)
{
    double mu[3] = {mean[0], mean[1], mean[2]};
    double p[3];
    for (int r = 0; r < 3; ++r)
        p[r] = cam->R_wc[r * 3 + 0] * mu[0] + cam->R_wc[r * 3 + 1] * mu[1] +
               cam->R_wc[r * 3 + 2] * mu[2] + cam->t_wc[r];
    double z = p[2];
    P->z = z;
    P->in_front = z > near;
    P->near_marginal = fabs(z - near) <= eps_near;
    if (!P->in_front && !P->near_marginal) return 0;
    if (z <= 0.0) return 0;

    /* Sigma = R S S^T R^T */
    double q[4] = {quat[0], quat[1], quat[2], quat[3]};
    double Rq[9];
    gso_quat_to_rot(q, Rq);
    double s2[3] = {(double)scale[0] * scale[0], (double)scale[1] * scale[1],
                    (double)scale[2] * scale[2]};
    double Sig[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0;
            for (int k = 0; k < 3; ++k) a += Rq[i * 3 + k] * s2[k] * Rq[j * 3 + k];
            Sig[i * 3 + j] = a;
        }

    /* J at the clamped tangent; Sigma' = J W Sigma W^T J^T + 0.3 I */
    double xz = p[0] / z, yz = p[1] / z;
    double lxn = -TAN_CLAMP * cam->cx / cam->fx, lxp = TAN_CLAMP * (cam->W - cam->cx) / cam->fx;
    double lyn = -TAN_CLAMP * cam->cy / cam->fy, lyp = TAN_CLAMP * (cam->H - cam->cy) / cam->fy;
    double tx = fmin(fmax(xz, lxn), lxp), ty = fmin(fmax(yz, lyn), lyp);
    double J[6] = {cam->fx / z, 0.0, -cam->fx * tx / z,
                   0.0, cam->fy / z, -cam->fy * ty / z};
    double T[6]; /* T = J W  (2x3) */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double a = 0;
            for (int k = 0; k < 3; ++k) a += J[r * 3 + k] * cam->R_wc[k * 3 + c];
            T[r * 3 + c] = a;
        }
    double M[4]; /* T Sigma T^T */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double a = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) a += T[r * 3 + i] * Sig[i * 3 + j] * T[c * 3 + j];
            M[r * 2 + c] = a;
        }
    double a = M[0] + LOWPASS, b = 0.5 * (M[1] + M[2]), c = M[3] + LOWPASS;
    double det = a * c - b * b;
    P->cov[0] = a; P->cov[1] = b; P->cov[2] = c;
    P->conic[0] = c / det; P->conic[1] = -b / det; P->conic[2] = a / det;
    P->u = cam->fx * p[0] / z + cam->cx;
    P->v = cam->fy * p[1] / z + cam->cy;
    P->o = opacity;

    /* colour from SH along the camera-centre -> mean direction (world) */
    double d[3] = {mu[0] - cam->C[0], mu[1] - cam->C[1], mu[2] - cam->C[2]};
    int ncoef = (deg + 1) * (deg + 1);
    double coef[48];
    for (int k = 0; k < ncoef * 3; ++k) coef[k] = sh[k];
    gso_sh_color(deg, d, coef, P->rgb);
    return 1;
}

/* pixel-centre range {i : |i + 1/2 - centre| <= ext} clipped to [0, n-1] */
static void centre_range(double centre, double ext, int n, int *lo, int *hi)
{
    double a = ceil(centre - ext - 0.5), b = floor(centre + ext - 0.5);
    if (a < 0) a = 0;
    if (b > n - 1) b = n - 1;
    if (a > b) { *lo = 1; *hi = 0; return; }
    *lo = (int)a; *hi = (int)b;
}

/* Fill the exact footprint box (alpha >= ALPHA_MIN) and the padded box used
 * to collect candidates (alpha >= ALPHA_MIN (1 - eps_alpha), one extra pixel
 * on every side). Returns 1 if the padded box is non-empty. */
static int footprint(proj_t *P, int W, int H, double eps_alpha, int *bx0, int *bx1,
                     int *by0, int *by1)
{
    P->hits_image = 0;
    P->x0 = 1; P->x1 = 0; P->y0 = 1; P->y1 = 0;
    if (P->o >= ALPHA_MIN) {
        double r2 = 2.0 * log(P->o / ALPHA_MIN);
        centre_range(P->u, sqrt(r2 * P->cov[0]), W, &P->x0, &P->x1);
        centre_range(P->v, sqrt(r2 * P->cov[2]), H, &P->y0, &P->y1);
        P->hits_image = P->x0 <= P->x1 && P->y0 <= P->y1;
    }
    double amin = ALPHA_MIN * (1.0 - eps_alpha);
    if (P->o < amin) return 0;
    double r2 = 2.0 * log(P->o / amin);
    centre_range(P->u, sqrt(r2 * P->cov[0]) + 1.0, W, bx0, bx1);
    centre_range(P->v, sqrt(r2 * P->cov[2]) + 1.0, H, by0, by1);
    return *bx0 <= *bx1 && *by0 <= *by1;
}

/* Projection of every Gaussian; out[g*20 ...] = u, v, z, cov a b c,
 * conic A B C, o, r, g, b, x0, x1, y0, y1, in_front, hits_image, projected. */
void gso_project_all(const float *means, const float *scales, const float *quats,
                     const float *opacity, const float *sh, int64_t n, int deg,
                     const float pose[12], const float intr[4], int W, int H,
                     double near, double *out)
{
    camera_t cam;
    camera_setup(pose, intr, W, H, &cam);
    int ncoef = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        proj_t P;
        memset(&P, 0, sizeof P);
        double *o = out + g * 20;
        int ok = project_one(&cam, means + g * 3, scales + g * 3, quats + g * 4,
                             opacity[g], sh + g * ncoef * 3, deg, near, 0.0, &P);
        int bx0, bx1, by0, by1;
        if (ok && P.in_front) footprint(&P, W, H, 0.0, &bx0, &bx1, &by0, &by1);
        o[0] = P.u; o[1] = P.v; o[2] = P.z;
        o[3] = P.cov[0]; o[4] = P.cov[1]; o[5] = P.cov[2];
        o[6] = P.conic[0]; o[7] = P.conic[1]; o[8] = P.conic[2];
        o[9] = P.o; o[10] = P.rgb[0]; o[11] = P.rgb[1]; o[12] = P.rgb[2];
        o[13] = P.x0; o[14] = P.x1; o[15] = P.y0; o[16] = P.y1;
        o[17] = ok && P.in_front;
        o[18] = ok && P.in_front && P.hits_image;
        o[19] = ok;
    }
}

/* ------------------------------------------------------------ compositing -- */

typedef struct {
    int x;
    int32_t g;
    double z, alpha, rgb[3];
    int near_marginal, in_front;
} cand_t;

static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = pa, *b = pb;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->z != b->z) return a->z < b->z ? -1 : 1;
    return (a->g > b->g) - (a->g < b->g);
}

typedef struct {
    double bg[3];
    double eps_alpha, eps_T;
    int max_leaves;
} walk_cfg_t;

#define MAX_LEAVES 1024

typedef struct {
    int n;
    int overflow;
    double v[MAX_LEAVES][5];
} leaves_t;

static void emit_leaf(leaves_t *L, const walk_cfg_t *cfg, double T, const double acc[5])
{
    if (L->n >= cfg->max_leaves || L->n >= MAX_LEAVES) { L->overflow = 1; return; }
    double *v = L->v[L->n++];
    v[0] = acc[0] + T * cfg->bg[0];
    v[1] = acc[1] + T * cfg->bg[1];
    v[2] = acc[2] + T * cfg->bg[2];
    v[3] = acc[4] > 0 ? acc[3] / acc[4] : 0.0;
    v[4] = acc[4];
}

/* Outcome of one candidate in the walk of step 6. */
enum { OUT_PASS = 0, OUT_STOP = 1, OUT_ACC = 2 };

static int outcome(const cand_t *k, double T, int present, int skip_flip, int stop_flip)
{
    if (!present) return OUT_PASS;
    int skip = k->alpha < ALPHA_MIN;
    if (skip_flip) skip = !skip;
    if (skip) return OUT_PASS;
    int stop = T * (1.0 - k->alpha) < T_MIN;
    if (stop_flip) stop = !stop;
    return stop ? OUT_STOP : OUT_ACC;
}

/* Step 6 where every decision that sits within its margin (near plane,
 * skip at ALPHA_MIN, stop at T_MIN) is taken both ways; each complete walk
 * emits one leaf. The natural FP64 decision is followed in the loop, the
 * alternatives by recursion. */
static void walk_branching(const cand_t *c, const int *order, int n, int i, double T,
                           const double acc_in[5], const walk_cfg_t *cfg, leaves_t *L)
{
    double acc[5];
    memcpy(acc, acc_in, sizeof acc);
    for (; i < n; ++i) {
        const cand_t *k = &c[order[i]];
        int m_near = k->near_marginal;
        int m_skip = fabs(k->alpha - ALPHA_MIN) <= cfg->eps_alpha * ALPHA_MIN;
        int m_stop = fabs(T * (1.0 - k->alpha) - T_MIN) <= cfg->eps_T * T_MIN;
        int natural = outcome(k, T, k->in_front, 0, 0);
        int seen = 1 << natural;
        for (int f = 1; f < 8; ++f) {
            if (((f & 1) && !m_near) || ((f & 2) && !m_skip) || ((f & 4) && !m_stop)) continue;
            int present = (f & 1) ? !k->in_front : k->in_front;
            int alt = outcome(k, T, present, (f >> 1) & 1, (f >> 2) & 1);
            if (seen >> alt & 1) continue;
            seen |= 1 << alt;
            if (alt == OUT_PASS) {
                walk_branching(c, order, n, i + 1, T, acc, cfg, L);
            } else if (alt == OUT_STOP) {
                emit_leaf(L, cfg, T, acc);
            } else {
                double acc2[5];
                double w = k->alpha * T;
                acc2[0] = acc[0] + w * k->rgb[0]; acc2[1] = acc[1] + w * k->rgb[1];
                acc2[2] = acc[2] + w * k->rgb[2]; acc2[3] = acc[3] + w * k->z;
                acc2[4] = acc[4] + w;
                walk_branching(c, order, n, i + 1, T * (1.0 - k->alpha), acc2, cfg, L);
            }
        }
        if (natural == OUT_PASS) continue;
        if (natural == OUT_STOP) { emit_leaf(L, cfg, T, acc); return; }
        double w = k->alpha * T;
        acc[0] += w * k->rgb[0]; acc[1] += w * k->rgb[1]; acc[2] += w * k->rgb[2];
        acc[3] += w * k->z; acc[4] += w;
        T = T * (1.0 - k->alpha);
    }
    emit_leaf(L, cfg, T, acc);
}

/* Near-tie runs: at most MAX_RUNS runs of at most MAX_RUN_LEN members and
 * MAX_ORDERS orders in all per pixel (else the pixel is unresolved). */
#define MAX_RUNS 8
#define MAX_RUN_LEN 4
#define MAX_ORDERS 256

/* Rearrange p[0..len) into its k-th permutation in lexicographic order
 * (k < len!, decoded as a factorial-base number). */
static void run_order(int *p, int len, long k)
{
    int pool[MAX_RUN_LEN], out[MAX_RUN_LEN];
    for (int i = 0; i < len; ++i) pool[i] = p[i];
    int left = len;
    for (int i = 0; i < len; ++i) {
        long f = (long)factorial(len - 1 - i);
        int sel = (int)(k / f);
        k %= f;
        out[i] = pool[sel];
        for (int j = sel; j + 1 < left; ++j) pool[j] = pool[j + 1];
        --left;
    }
    for (int i = 0; i < len; ++i) p[i] = out[i];
}

/* Step 6 with the natural FP64 decisions only. Returns the contributor count;
 * *reach is the number of candidates the walk examined (the stopping one
 * included). */
static int walk_plain(const cand_t *c, int n, const walk_cfg_t *cfg, double out[5],
                      double *T_out, int *marginal, int *reach)
{
    double T = 1.0, acc[5] = {0, 0, 0, 0, 0};
    int ncontrib = 0;
    *marginal = 0;
    *reach = n;
    for (int i = 0; i < n; ++i) {
        const cand_t *k = &c[i];
        if (k->near_marginal) *marginal = 1;
        if (!k->in_front) continue;
        double a = k->alpha;
        if (fabs(a - ALPHA_MIN) <= cfg->eps_alpha * ALPHA_MIN) *marginal = 1;
        if (a < ALPHA_MIN) continue;
        double Tn = T * (1.0 - a);
        if (fabs(Tn - T_MIN) <= cfg->eps_T * T_MIN) *marginal = 1;
        if (Tn < T_MIN) {
            *reach = i + 1;
            break;
        }
        double w = a * T;
        acc[0] += w * k->rgb[0]; acc[1] += w * k->rgb[1]; acc[2] += w * k->rgb[2];
        acc[3] += w * k->z; acc[4] += w;
        T = Tn;
        ++ncontrib;
    }
    out[0] = acc[0] + T * cfg->bg[0];
    out[1] = acc[1] + T * cfg->bg[1];
    out[2] = acc[2] + T * cfg->bg[2];
    out[3] = acc[4] > 0 ? acc[3] / acc[4] : 0.0;
    out[4] = acc[4];
    *T_out = T;
    return ncontrib;
}

/*
 * Render one camera.
 *
 * Inputs: FP32 scene arrays (means [n][3], scales [n][3] linear, quats [n][4]
 * (w,x,y,z), opacity [n], sh [n][(deg+1)^2][3]), pose [3][4] camera-to-world,
 * intrinsics (fx, fy, cx, cy), image W x H, near plane, background,
 * margins[4] = (eps_alpha relative, eps_T relative, eps_z absolute metres,
 * eps_near absolute metres).
 *
 * Outputs (FP64, caller-allocated): rgb [H][W][3], depth [H][W], alpha
 * [H][W], tfinal [H][W] (transmittance after the walk); counters[8] =
 * projected, visible (exact box hits a pixel centre), instances for 16x16
 * tiles over the exact boxes, contributing pairs P, flagged pixels,
 * unresolved pixels (too many alternatives), candidate pairs, variants.
 * For flagged pixels the alternative results go to var_pix[k] (pixel index
 * y*W+x) and var_vals[k][5] = (r, g, b, depth, alpha) while k < var_cap (an
 * unresolved pixel gets one entry of NaNs: it has alternatives, none known);
 * *n_var receives the number of alternatives produced (may exceed var_cap).
 */
int gso_render(const float *means, const float *scales, const float *quats,
               const float *opacity, const float *sh, int64_t n, int deg,
               const float pose[12], const float intr[4], int W, int H, double near,
               const double bg[3], const double margins[4], double *rgb,
               double *depth, double *alpha, double *tfinal, int64_t *counters,
               int64_t var_cap, int32_t *var_pix, double *var_vals, int64_t *n_var,
               int nthreads)
{
    if (W <= 0 || H <= 0 || n < 0 || deg < 0 || deg > 3) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    camera_t cam;
    camera_setup(pose, intr, W, H, &cam);
    int ncoef = (deg + 1) * (deg + 1);
    double eps_alpha = margins[0], eps_T = margins[1], eps_z = margins[2],
           eps_near = margins[3];

    proj_t *P = (proj_t *)malloc(sizeof(proj_t) * (size_t)(n > 0 ? n : 1));
    int32_t *pb = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(n > 0 ? n : 1));
    char *live = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t n_proj = 0, n_vis = 0, n_inst = 0;

#pragma omp parallel for schedule(static) reduction(+ : n_proj, n_vis, n_inst)
    for (int64_t g = 0; g < n; ++g) {
        if (!project_one(&cam, means + g * 3, scales + g * 3, quats + g * 4, opacity[g],
                         sh + g * ncoef * 3, deg, near, eps_near, &P[g]))
            continue;
        int x0, x1, y0, y1;
        if (!footprint(&P[g], W, H, eps_alpha, &x0, &x1, &y0, &y1)) continue;
        live[g] = 1;
        pb[g * 4 + 0] = x0; pb[g * 4 + 1] = x1; pb[g * 4 + 2] = y0; pb[g * 4 + 3] = y1;
        if (P[g].in_front) {
            ++n_proj;
            if (P[g].hits_image) {
                ++n_vis;
                n_inst += (int64_t)(P[g].x1 / 16 - P[g].x0 / 16 + 1) *
                          (P[g].y1 / 16 - P[g].y0 / 16 + 1);
            }
        }
    }

    /* rows -> Gaussians whose padded box spans the row (CSR) */
    int64_t *row_start = (int64_t *)calloc((size_t)H + 1, sizeof(int64_t));
    for (int64_t g = 0; g < n; ++g)
        if (live[g])
            for (int y = pb[g * 4 + 2]; y <= pb[g * 4 + 3]; ++y) row_start[y + 1]++;
    for (int y = 0; y < H; ++y) row_start[y + 1] += row_start[y];
    int32_t *row_g = (int32_t *)malloc(sizeof(int32_t) * (size_t)(row_start[H] > 0 ? row_start[H] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
    for (int y = 0; y < H; ++y) fill[y] = row_start[y];
    for (int64_t g = 0; g < n; ++g)
        if (live[g])
            for (int y = pb[g * 4 + 2]; y <= pb[g * 4 + 3]; ++y) row_g[fill[y]++] = (int32_t)g;

    walk_cfg_t cfg = {{bg[0], bg[1], bg[2]}, eps_alpha, eps_T, MAX_LEAVES};
    int64_t n_pairs = 0, n_flag = 0, n_unres = 0, n_cand = 0, var_count = 0;

#pragma omp parallel reduction(+ : n_pairs, n_flag, n_unres, n_cand)
    {
        size_t cap = 1024;
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * cap);
        int *order = (int *)malloc(sizeof(int) * 4096);
        int order_cap = 4096;
        leaves_t *L = (leaves_t *)malloc(sizeof(leaves_t));
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < H; ++y) {
            size_t m = 0;
            double py = y + 0.5;
            for (int64_t e = row_start[y]; e < row_start[y + 1]; ++e) {
                int32_t g = row_g[e];
                const proj_t *q = &P[g];
                for (int x = pb[g * 4 + 0]; x <= pb[g * 4 + 1]; ++x) {
                    double dx = x + 0.5 - q->u, dy = py - q->v;
                    double power = -0.5 * (q->conic[0] * dx * dx + 2.0 * q->conic[1] * dx * dy +
                                           q->conic[2] * dy * dy);
                    double a = fmin(ALPHA_MAX, q->o * exp(power));
                    if (a < ALPHA_MIN * (1.0 - eps_alpha)) continue;
                    if (m == cap) {
                        cap *= 2;
                        buf = (cand_t *)realloc(buf, sizeof(cand_t) * cap);
                    }
                    cand_t *c = &buf[m++];
                    c->x = x; c->g = g; c->z = q->z; c->alpha = a;
                    c->rgb[0] = q->rgb[0]; c->rgb[1] = q->rgb[1]; c->rgb[2] = q->rgb[2];
                    c->near_marginal = q->near_marginal; c->in_front = q->in_front;
                }
            }
            qsort(buf, m, sizeof(cand_t), cand_cmp);
            size_t s = 0;
            for (int x = 0; x < W; ++x) {
                size_t e = s;
                while (e < m && buf[e].x == x) ++e;
                const cand_t *c = buf + s;
                int cn = (int)(e - s);
                int64_t pix = (int64_t)y * W + x;
                double out[5], T;
                int marginal, reach;
                int nc = walk_plain(c, cn, &cfg, out, &T, &marginal, &reach);
                for (int i = 0; i < cn; ++i) n_cand += c[i].in_front && c[i].alpha >= ALPHA_MIN;
                n_pairs += nc;
                rgb[pix * 3 + 0] = out[0]; rgb[pix * 3 + 1] = out[1]; rgb[pix * 3 + 2] = out[2];
                depth[pix] = out[3]; alpha[pix] = out[4]; tfinal[pix] = T;
                /* Runs of near-tied depths in the (z, index) order (consecutive
                 * gaps within eps_z) that start among the candidates the walk
                 * reaches: every order of such a run is a correct result, since
                 * rounding may order its members either way. Past the stop, any
                 * reordering changes the pixel by less than the final
                 * transmittance (< 1e-4 times the largest colour). */
                int run_s[MAX_RUNS], run_n[MAX_RUNS], nr = 0, unres = 0;
                long n_orders = 1;
                for (int i = 0; i + 1 < cn && i < reach;) {
                    if (!(fabs(c[i + 1].z - c[i].z) <= eps_z)) { ++i; continue; }
                    int j = i + 1;
                    while (j + 1 < cn && fabs(c[j + 1].z - c[j].z) <= eps_z) ++j;
                    if (j - i + 1 > MAX_RUN_LEN || nr == MAX_RUNS) {
                        unres = 1;
                    } else {
                        run_s[nr] = i;
                        run_n[nr] = j - i + 1;
                        n_orders *= (long)factorial(run_n[nr]);
                        ++nr;
                    }
                    i = j + 1;
                }
                if (!marginal && nr == 0 && !unres) { s = e; continue; }
                ++n_flag;
                if (unres || n_orders > MAX_ORDERS) {
                    /* no alternative can be listed: one entry of NaNs marks
                     * the pixel as not plain, and matches nothing */
                    ++n_unres;
                    int64_t base;
#pragma omp atomic capture
                    { base = var_count; var_count += 1; }
                    if (base < var_cap) {
                        var_pix[base] = (int32_t)pix;
                        for (int q = 0; q < 5; ++q) var_vals[base * 5 + q] = NAN;
                    }
                    s = e;
                    continue;
                }
                if (cn > order_cap) {
                    order_cap = cn * 2;
                    order = (int *)realloc(order, sizeof(int) * order_cap);
                }
                L->n = 0; L->overflow = 0;
                for (long k = 0; k < n_orders; ++k) {
                    for (int i = 0; i < cn; ++i) order[i] = i;
                    long rem = k;
                    for (int r = 0; r < nr; ++r) {
                        long f = (long)factorial(run_n[r]);
                        run_order(order + run_s[r], run_n[r], rem % f);
                        rem /= f;
                    }
                    double acc0[5] = {0, 0, 0, 0, 0};
                    walk_branching(c, order, cn, 0, 1.0, acc0, &cfg, L);
                }
                if (L->overflow) ++n_unres;
                int64_t base;
#pragma omp atomic capture
                { base = var_count; var_count += L->n; }
                for (int k = 0; k < L->n; ++k)
                    if (base + k < var_cap) {
                        var_pix[base + k] = (int32_t)pix;
                        memcpy(var_vals + (base + k) * 5, L->v[k], 5 * sizeof(double));
                    }
                s = e;
            }
        }
        free(buf);
        free(order);
        free(L);
    }
    counters[0] = n_proj; counters[1] = n_vis; counters[2] = n_inst;
    counters[3] = n_pairs; counters[4] = n_flag; counters[5] = n_unres;
    counters[6] = n_cand; counters[7] = var_count;
    *n_var = var_count;
    free(P); free(pb); free(live); free(row_start); free(row_g); free(fill);
    return 0;
}

/*
 * Diagnostic: the (z, index)-ordered candidates of one pixel (i, j) with
 * alpha >= ALPHA_MIN (1 - eps_alpha), for inspecting decisions near a
 * threshold. out[k*6 ...] = g, z, alpha, T before, T after, flags (1 near
 * marginal, 2 not in front). Returns the number of candidates (at most cap
 * are written).
 */
int gso_pixel_trace(const float *means, const float *scales, const float *quats,
                    const float *opacity, const float *sh, int64_t n, int deg,
                    const float pose[12], const float intr[4], int W, int H, double near,
                    double eps_alpha, int i, int j, int cap, double *out)
{
    camera_t cam;
    camera_setup(pose, intr, W, H, &cam);
    int ncoef = (deg + 1) * (deg + 1);
    int m = 0, mcap = 1024;
    cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * mcap);
    for (int64_t g = 0; g < n; ++g) {
        proj_t P;
        if (!project_one(&cam, means + g * 3, scales + g * 3, quats + g * 4, opacity[g],
                         sh + g * ncoef * 3, deg, near, 1e-5, &P))
            continue;
        double dx = i + 0.5 - P.u, dy = j + 0.5 - P.v;
        double power = -0.5 * (P.conic[0] * dx * dx + 2.0 * P.conic[1] * dx * dy +
                               P.conic[2] * dy * dy);
        double a = fmin(ALPHA_MAX, P.o * exp(power));
        if (a < ALPHA_MIN * (1.0 - eps_alpha)) continue;
        if (m == mcap) { mcap *= 2; buf = (cand_t *)realloc(buf, sizeof(cand_t) * mcap); }
        cand_t *c = &buf[m++];
        c->x = i; c->g = (int32_t)g; c->z = P.z; c->alpha = a;
        c->rgb[0] = P.rgb[0]; c->rgb[1] = P.rgb[1]; c->rgb[2] = P.rgb[2];
        c->near_marginal = P.near_marginal; c->in_front = P.in_front;
    }
    qsort(buf, m, sizeof(cand_t), cand_cmp);
    double T = 1.0;
    for (int k = 0; k < m && k < cap; ++k) {
        double Tn = T * (1.0 - buf[k].alpha);
        out[k * 6 + 0] = buf[k].g; out[k * 6 + 1] = buf[k].z; out[k * 6 + 2] = buf[k].alpha;
        out[k * 6 + 3] = T; out[k * 6 + 4] = Tn;
        out[k * 6 + 5] = buf[k].near_marginal + 2 * !buf[k].in_front;
        if (buf[k].in_front && buf[k].alpha >= ALPHA_MIN && !(Tn < T_MIN)) T = Tn;
    }
    free(buf);
    return m;
}
