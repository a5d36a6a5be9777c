/*
 * Plain FP64 CPU oracle for fast high-dimensional bilateral / nonlocal-means
 * filtering (Nair & Chaudhury, "Fast High-Dimensional Bilateral and Nonlocal
 * Means Filtering").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code with the
 * GPU library: it is written directly from the paper's definitions, with no
 * tiling, fusion or reordering beyond what a definition states.
 *
 * Layout of every image argument: planar (C, H, W), row-major, FP64.
 * Boundary reading: window samples that fall outside the image domain are
 * excluded from both sums (equivalently, the convolved images are
 * zero-extended).  Kernels are unnormalised (peak value 1).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the OpenMP loops below (the CPU baseline times one thread as
 * well as all of them). */
void oracle_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

/* Spatial kernel, Sec. III: Gaussian exp(-|j|^2 / 2 sigma_s^2) for the
 * bilateral filter, box (weight 1) for nonlocal means. */
static double omega2(int jy, int jx, int spatial, double sigma_s)
{
    if (spatial == 1) return 1.0;
    return exp(-(double)(jy * jy + jx * jx) / (2.0 * sigma_s * sigma_s));
}

static double omega1(int t, int spatial, double sigma_s)
{
    if (spatial == 1) return 1.0;
    return exp(-(double)(t * t) / (2.0 * sigma_s * sigma_s));
}

/* Table of the 2-D spatial kernel over the window, indexed
 * [(jy + S) * (2S+1) + (jx + S)]. */
static double *omega_table(int S, int spatial, double sigma_s)
{
    const int L = 2 * S + 1;
    double *t = (double *)malloc(sizeof(double) * (size_t)L * (size_t)L);
    for (int jy = -S; jy <= S; ++jy)
        for (int jx = -S; jx <= S; ++jx)
            t[(jy + S) * L + (jx + S)] = omega2(jy, jx, spatial, sigma_s);
    return t;
}

/* Range kernel, Sec. III: isotropic Gaussian of the squared distance.
 * sigma_r = +inf gives phi == 1. */
static double phi(double d2, double sigma_r)
{
    if (isinf(sigma_r)) return 1.0;
    return exp(-d2 / (2.0 * sigma_r * sigma_r));
}

/* Brute-force filter, eqs. (1)-(2): for every pixel i,
 *   g(i) = sum_j w(j) phi(p(i-j) - p(i)) f(i-j) / eta(i),
 *   eta(i) = sum_j w(j) phi(p(i-j) - p(i)),  j in [-S, S]^2, i-j in Omega.
 * den (may be NULL) receives eta. */
void oracle_bruteforce(const double *f, int n, const double *p, int rho,
                       int H, int W, int S, int spatial, double sigma_s,
                       double sigma_r, double *out, double *den)
{
    const long N = (long)H * W;
    double *wt = omega_table(S, spatial, sigma_s);
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y) {
        double *num = (double *)malloc(sizeof(double) * (size_t)n);
        for (int x = 0; x < W; ++x) {
            const long i = (long)y * W + x;
            double eta = 0.0;
            for (int c = 0; c < n; ++c) num[c] = 0.0;
            for (int jy = -S; jy <= S; ++jy) {
                const int yy = y - jy;
                if (yy < 0 || yy >= H) continue;
                for (int jx = -S; jx <= S; ++jx) {
                    const int xx = x - jx;
                    if (xx < 0 || xx >= W) continue;
                    const long q = (long)yy * W + xx;
                    double d2 = 0.0;
                    for (int r = 0; r < rho; ++r) {
                        const double t = p[r * N + q] - p[r * N + i];
                        d2 += t * t;
                    }
                    const double w = wt[(jy + S) * (2 * S + 1) + (jx + S)] * phi(d2, sigma_r);
                    for (int c = 0; c < n; ++c) num[c] += w * f[c * N + q];
                    eta += w;
                }
            }
            for (int c = 0; c < n; ++c) out[c * N + i] = num[c] / eta;
            if (den) den[i] = eta;
        }
        free(num);
    }
    free(wt);
}

/* Brute force (eqs. (1)-(2)) evaluated only at the M pixels (ys[m], xs[m]).
 * out is M x n, den is M (may be NULL). */
void oracle_bruteforce_at(const double *f, int n, const double *p, int rho,
                          int H, int W, int S, int spatial, double sigma_s,
                          double sigma_r, const int *ys, const int *xs, int M,
                          double *out, double *den)
{
    const long N = (long)H * W;
    double *wt = omega_table(S, spatial, sigma_s);
#pragma omp parallel for schedule(dynamic, 4)
    for (int m = 0; m < M; ++m) {
        const int y = ys[m], x = xs[m];
        const long i = (long)y * W + x;
        double eta = 0.0;
        double *num = out + (long)m * n;
        for (int c = 0; c < n; ++c) num[c] = 0.0;
        for (int jy = -S; jy <= S; ++jy) {
            const int yy = y - jy;
            if (yy < 0 || yy >= H) continue;
            for (int jx = -S; jx <= S; ++jx) {
                const int xx = x - jx;
                if (xx < 0 || xx >= W) continue;
                const long q = (long)yy * W + xx;
                double d2 = 0.0;
                for (int r = 0; r < rho; ++r) {
                    const double t = p[r * N + q] - p[r * N + i];
                    d2 += t * t;
                }
                const double w = wt[(jy + S) * (2 * S + 1) + (jx + S)] * phi(d2, sigma_r);
                for (int c = 0; c < n; ++c) num[c] += w * f[c * N + q];
                eta += w;
            }
        }
        for (int c = 0; c < n; ++c) num[c] /= eta;
        if (den) den[m] = eta;
    }
    free(wt);
}

/* Linear convolution with the spatial kernel, as used in eqs. (13)-(14):
 *   v(i) = sum_{j in [-S,S]^2, i-j in Omega} w(j) u(i-j),
 * written as the direct two-dimensional window sum.  C planes. */
void oracle_conv2d(const double *u, int C, int H, int W, int S, int spatial,
                   double sigma_s, double *v)
{
    const long N = (long)H * W;
    double *wt = omega_table(S, spatial, sigma_s);
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int c = 0; c < C; ++c) {
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int jy = -S; jy <= S; ++jy) {
                    const int yy = y - jy;
                    if (yy < 0 || yy >= H) continue;
                    for (int jx = -S; jx <= S; ++jx) {
                        const int xx = x - jx;
                        if (xx < 0 || xx >= W) continue;
                        acc += wt[(jy + S) * (2 * S + 1) + (jx + S)] * u[c * N + (long)yy * W + xx];
                    }
                }
                v[c * N + (long)y * W + x] = acc;
            }
        }
    }
    free(wt);
}

/* The same convolution computed as a horizontal then a vertical 1-D pass.
 * Both spatial kernels factor into 1-D kernels: the Gaussian of |j|^2 is the
 * product of two 1-D Gaussians and the box is the product of two 1-D boxes,
 * and a zero-extended image stays zero-extended after the first pass.
 * Used where the direct sum is too slow (full-size images). */
void oracle_conv_separable(const double *u, int C, int H, int W, int S,
                           int spatial, double sigma_s, double *v)
{
    const long N = (long)H * W;
    double *w1 = (double *)malloc(sizeof(double) * (size_t)(2 * S + 1));
    for (int t = -S; t <= S; ++t) w1[t + S] = omega1(t, spatial, sigma_s);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N * (size_t)C);
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < C; ++c) {
        for (int y = 0; y < H; ++y) {
            const double *row = u + c * N + (long)y * W;
            double *trow = tmp + c * N + (long)y * W;
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int j = -S; j <= S; ++j) {
                    const int xx = x - j;
                    if (xx < 0 || xx >= W) continue;
                    acc += w1[j + S] * row[xx];
                }
                trow[x] = acc;
            }
        }
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < C; ++c) {
        for (int y = 0; y < H; ++y) {
            double *vrow = v + c * N + (long)y * W;
            for (int x = 0; x < W; ++x) vrow[x] = 0.0;
            for (int j = -S; j <= S; ++j) {
                const int yy = y - j;
                if (yy < 0 || yy >= H) continue;
                const double *trow = tmp + c * N + (long)yy * W;
                const double wj = w1[j + S];
                for (int x = 0; x < W; ++x) vrow[x] += wj * trow[x];
            }
        }
    }
    free(tmp);
    free(w1);
}

/* The cluster images of eqs. (13)-(14) evaluated only at the M pixels
 * (ys[m], xs[m]) for the K centers mu (K x rho):
 *   V[m][k][c] = sum_j w(j) phi(p(i-j) - mu_k) f_c(i-j)   for c < n,
 *   V[m][k][n] = sum_j w(j) phi(p(i-j) - mu_k)             (r_k of eq. (14)).
 * V is M x K x (n+1). */
void oracle_cluster_images_at(const double *f, int n, const double *p, int rho,
                              int H, int W, const double *mu, int K, int S,
                              int spatial, double sigma_s, double sigma_r,
                              const int *ys, const int *xs, int M, double *V)
{
    const long N = (long)H * W;
    double *wt = omega_table(S, spatial, sigma_s);
#pragma omp parallel for schedule(dynamic, 1)
    for (int m = 0; m < M; ++m) {
        const int y = ys[m], x = xs[m];
        double *Vm = V + (long)m * K * (n + 1);
        for (int t = 0; t < K * (n + 1); ++t) Vm[t] = 0.0;
        for (int jy = -S; jy <= S; ++jy) {
            const int yy = y - jy;
            if (yy < 0 || yy >= H) continue;
            for (int jx = -S; jx <= S; ++jx) {
                const int xx = x - jx;
                if (xx < 0 || xx >= W) continue;
                const long q = (long)yy * W + xx;
                const double w = wt[(jy + S) * (2 * S + 1) + (jx + S)];
                for (int k = 0; k < K; ++k) {
                    double d2 = 0.0;
                    for (int r = 0; r < rho; ++r) {
                        const double t = p[r * N + q] - mu[k * rho + r];
                        d2 += t * t;
                    }
                    const double wb = w * phi(d2, sigma_r);
                    double *Vk = Vm + k * (n + 1);
                    for (int c = 0; c < n; ++c) Vk[c] += wb * f[c * N + q];
                    Vk[n] += wb;
                }
            }
        }
    }
    free(wt);
}
