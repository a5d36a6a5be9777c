// The K x K least-squares solve of Algorithm 1 (eqs. (11)-(12)): the kernel
// matrix A_kl = phi(mu_k - mu_l) and its Moore-Penrose pseudo-inverse, in FP64
// on the host, and the symmetric eigen-decomposition it uses (also used for the
// patch covariance of the nonlocal-means guide).  A is symmetric, so its
// singular values are |eigenvalues| and A^+ = sum over kept eigenpairs of
// v v^T / lambda.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fhd_internal.h"

namespace fhd {

void kernel_matrix(const float* centers, int K, int rho, double sigma_r, double* A) {
    const bool flat = std::isinf(sigma_r);
    const double inv = flat ? 0.0 : 1.0 / (2.0 * sigma_r * sigma_r);
    for (int k = 0; k < K; ++k) {
        A[(size_t)k * K + k] = 1.0;
        for (int l = k + 1; l < K; ++l) {
            double d2 = 0.0;
            for (int t = 0; t < rho; ++t) {
                const double d = (double)centers[(size_t)k * rho + t] - (double)centers[(size_t)l * rho + t];
                d2 += d * d;
            }
            const double v = flat ? 1.0 : std::exp(-d2 * inv);
            A[(size_t)k * K + l] = v;
            A[(size_t)l * K + k] = v;
        }
    }
}

// Eigen-decomposition of a symmetric n x n matrix (row-major, destroyed):
// Householder reduction to tridiagonal form, then implicit symmetric QR steps
// with the Wilkinson shift, the Givens rotations applied to the band of the
// tridiagonal matrix (plus its one-element bulge) and accumulated into the
// orthogonal factor.  On return lam[i] are the eigenvalues and column i of v
// (row-major n x n) the corresponding unit eigenvectors (unsorted).  Returns
// false when the off-diagonal band has not vanished after 64 n QR steps (a
// matrix with non-finite entries never converges); the caller then rejects
// the result.
// sqrt(a^2 + b^2) without the cost of std::hypot; the library's matrices
// (kernel matrices, covariances) stay far from overflow, hypot covers the rest
static inline double norm2(double a, double b) {
    const double m = std::max(std::fabs(a), std::fabs(b));
    return m < 1e150 && (m == 0.0 || m > 1e-150) ? std::sqrt(a * a + b * b) : std::hypot(a, b);
}

bool sym_eigen(std::vector<double>& t, int n, std::vector<double>& lam, std::vector<double>& v) {
    auto T = [&](int i, int j) -> double& { return t[(size_t)i * n + j]; };
    // the orthogonal factor is accumulated transposed (row c = column c of
    // the factor) so that every update runs along contiguous memory
    std::vector<double> qt((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) qt[(size_t)i * n + i] = 1.0;
    auto Q = [&](int i, int j) -> double& { return qt[(size_t)j * n + i]; };
    // --- Householder: T <- H T H on the trailing block, Q <- Q H
    std::vector<double> x(n), p(n), q(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double xn = 0.0;
        for (int i = 0; i < m; ++i) {
            x[i] = T(k + 1 + i, k);
            xn += x[i] * x[i];
        }
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const double alpha = x[0] >= 0.0 ? -xn : xn;
        x[0] -= alpha;  // x is now the reflector v
        double vn = 0.0;
        for (int i = 0; i < m; ++i) vn += x[i] * x[i];
        if (vn == 0.0) continue;
        const double beta = 2.0 / vn;
        double vp = 0.0;
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += T(k + 1 + i, k + 1 + j) * x[j];
            p[i] = beta * s;
            vp += x[i] * p[i];
        }
        const double kk = vp / vn;
        for (int i = 0; i < m; ++i) q[i] = p[i] - kk * x[i];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) T(k + 1 + i, k + 1 + j) -= x[i] * q[j] + q[i] * x[j];
        T(k + 1, k) = T(k, k + 1) = alpha;
        for (int i = 1; i < m; ++i) T(k + 1 + i, k) = T(k, k + 1 + i) = 0.0;
        // Q <- Q H: columns k+1.. of Q (rows of qt) minus beta (Q x) x^T
        std::vector<double>& w = p;  // reused: w = beta Q x, over the n rows of Q
        std::fill(w.begin(), w.end(), 0.0);
        if ((int)w.size() < n) w.resize(n);
        for (int j = 0; j < m; ++j) {
            const double* qc = &qt[(size_t)(k + 1 + j) * n];
            const double xj = x[j];
            for (int r = 0; r < n; ++r) w[r] += qc[r] * xj;
        }
        for (int j = 0; j < m; ++j) {
            double* qc = &qt[(size_t)(k + 1 + j) * n];
            const double bx = beta * x[j];
            for (int r = 0; r < n; ++r) qc[r] -= w[r] * bx;
        }
    }
    // --- implicit symmetric QR with Wilkinson shifts
    const double eps = 0x1p-52;
    auto rot = [&](int k, int lo, int hi, double c, double s) {
        // T <- G^T T G, G = rotation in the (k, k+1) plane, G_kk = G_k+1,k+1 = c, G_k,k+1 = s
        const int j0 = std::max(lo, k - 1), j1 = std::min(hi, k + 2);
        for (int j = j0; j <= j1; ++j) {
            const double a = T(k, j), b = T(k + 1, j);
            T(k, j) = c * a - s * b;
            T(k + 1, j) = s * a + c * b;
        }
        for (int i = j0; i <= j1; ++i) {
            const double a = T(i, k), b = T(i, k + 1);
            T(i, k) = c * a - s * b;
            T(i, k + 1) = s * a + c * b;
        }
        double* qa = &qt[(size_t)k * n];
        double* qb = &qt[(size_t)(k + 1) * n];
        for (int r = 0; r < n; ++r) {
            const double a = qa[r], b = qb[r];
            qa[r] = c * a - s * b;
            qb[r] = s * a + c * b;
        }
    };
    int hi = n - 1, guard = 0;
    while (hi > 0 && guard < 64 * n) {
        if (std::fabs(T(hi, hi - 1)) <= eps * (std::fabs(T(hi - 1, hi - 1)) + std::fabs(T(hi, hi)))) {
            T(hi, hi - 1) = T(hi - 1, hi) = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(T(lo, lo - 1)) > eps * (std::fabs(T(lo - 1, lo - 1)) + std::fabs(T(lo, lo)))) --lo;
        if (lo > 0) T(lo, lo - 1) = T(lo - 1, lo) = 0.0;
        ++guard;
        const double dd = 0.5 * (T(hi - 1, hi - 1) - T(hi, hi));
        const double ee = T(hi, hi - 1);
        const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * norm2(dd, ee);
        const double mu = T(hi, hi) - ee * ee / den;
        double xx = T(lo, lo) - mu, zz = T(lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            const double r = norm2(xx, zz);
            const double c = r == 0.0 ? 1.0 : xx / r, s = r == 0.0 ? 0.0 : -zz / r;
            rot(k, lo, hi, c, s);
            if (k + 1 < hi) {
                xx = T(k + 1, k);
                zz = T(k + 2, k);
            }
        }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = T(i, i);
    v.resize((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[(size_t)i * n + j] = qt[(size_t)j * n + i];
    if (hi > 0) return false;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(lam[i])) return false;
    return true;
}

void sym_eigen_checked(std::vector<double>& t, int n, std::vector<double>& lam, std::vector<double>& v,
                       const char* what) {
    FHD_REQUIRE(sym_eigen(t, n, lam, v), FHD_ENUMERIC,
                std::string("eigen-decomposition of ") + what + " did not converge (non-finite entries?)");
}

PinvResult pinv_symmetric(const double* A, int K, double rtol, double* P) {
    std::vector<double> a(A, A + (size_t)K * K), lam, v;
    sym_eigen_checked(a, K, lam, v, "the kernel matrix A");
    double smax = 0.0;
    for (double x : lam) smax = std::max(smax, std::fabs(x));
    const double tol = (rtol > 0.0 ? rtol : (double)K * 0x1p-52) * smax;
    PinvResult r;
    double smin = smax;
    std::fill(P, P + (size_t)K * K, 0.0);
    for (int i = 0; i < K; ++i) {
        if (!(std::fabs(lam[i]) > tol)) continue;
        ++r.rank;
        smin = std::min(smin, std::fabs(lam[i]));
        const double inv = 1.0 / lam[i];
        for (int k = 0; k < K; ++k) {
            const double vk = v[(size_t)k * K + i] * inv;
            for (int l = 0; l < K; ++l) P[(size_t)k * K + l] += vk * v[(size_t)l * K + i];
        }
    }
    r.cond = r.rank > 0 ? smax / smin : INFINITY;
    for (size_t q = 0; q < (size_t)K * K; ++q) r.max_abs = std::max(r.max_abs, std::fabs(P[q]));
    return r;
}

// dA^+/dsigma_r for A_kl = exp(-|mu_k - mu_l|^2 / (2 sigma_r^2)), with the
// kept eigenpairs of A held fixed (the rank decision of pinv_symmetric).
// A^+ = F(A) with the spectral function g(lam) = 1/lam on kept eigenvalues
// and 0 on dropped ones, so dF = V (D o (V^T dA V)) V^T with the divided
// differences D_ij = (g(lam_i) - g(lam_j)) / (lam_i - lam_j) (g' on equal
// pairs): -1/(lam_i lam_j) for two kept, 1/(lam_i (lam_i - lam_j)) for kept i
// and dropped j, 0 for two dropped.  dA/dsigma_r = A o |mu_k - mu_l|^2 / sigma_r^3.
// The derivative of A^+ (symmetric A, the pseudo-inverse's rank held fixed)
// along a symmetric direction X: V (D o (V^T X V)) V^T with the divided
// differences D_ij of f(lambda) = 1/lambda on kept eigenvalues, 0 on dropped
// ones (kept-kept -1/(l_i l_j), kept-dropped 1/(l_i (l_i - l_j)), dropped-
// dropped 0).  D is symmetric, so the same map applied to dL/dA^+ gives
// dL/dA (the map is its own adjoint).
static void pinv_directional(const std::vector<double>& lam, const std::vector<double>& V,
                             const std::vector<char>& kept, int K, const double* X, double* Y) {
    std::vector<double> T((size_t)K * K, 0.0), E((size_t)K * K, 0.0);
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < K; ++j) {
            double s = 0.0;
            for (int l = 0; l < K; ++l) s += X[(size_t)k * K + l] * V[(size_t)l * K + j];
            T[(size_t)k * K + j] = s;
        }
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) {
            double s = 0.0;
            for (int k = 0; k < K; ++k) s += V[(size_t)k * K + i] * T[(size_t)k * K + j];
            double d;
            if (kept[i] && kept[j])
                d = -1.0 / (lam[i] * lam[j]);
            else if (kept[i])
                d = 1.0 / (lam[i] * (lam[i] - lam[j]));
            else if (kept[j])
                d = 1.0 / (lam[j] * (lam[j] - lam[i]));
            else
                d = 0.0;
            E[(size_t)i * K + j] = s * d;
        }
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < K; ++j) {
            double s = 0.0;
            for (int i = 0; i < K; ++i) s += V[(size_t)k * K + i] * E[(size_t)i * K + j];
            T[(size_t)k * K + j] = s;
        }
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) {
            double s = 0.0;
            for (int j = 0; j < K; ++j) s += T[(size_t)k * K + j] * V[(size_t)l * K + j];
            Y[(size_t)k * K + l] = s;
        }
}

// eigen-decomposition of A and the kept set of its pseudo-inverse
static void pinv_spectrum(const std::vector<double>& A, int K, double rtol, std::vector<double>& lam,
                          std::vector<double>& V, std::vector<char>& kept) {
    std::vector<double> t = A;
    sym_eigen_checked(t, K, lam, V, "the kernel matrix A");
    double smax = 0.0;
    for (double x : lam) smax = std::max(smax, std::fabs(x));
    const double tol = (rtol > 0.0 ? rtol : (double)K * 0x1p-52) * smax;
    kept.assign(K, 0);
    for (int i = 0; i < K; ++i) kept[i] = std::fabs(lam[i]) > tol;
}

void pinv_sigma_derivative(const float* centers, int K, int rho, double sigma_r, double rtol, double* M) {
    std::fill(M, M + (size_t)K * K, 0.0);
    if (std::isinf(sigma_r)) return;
    std::vector<double> A((size_t)K * K), dA((size_t)K * K);
    kernel_matrix(centers, K, rho, sigma_r, A.data());
    const double s3 = sigma_r * sigma_r * sigma_r;
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) {
            double d2 = 0.0;
            for (int t = 0; t < rho; ++t) {
                const double d = (double)centers[(size_t)k * rho + t] - (double)centers[(size_t)l * rho + t];
                d2 += d * d;
            }
            dA[(size_t)k * K + l] = A[(size_t)k * K + l] * d2 / s3;
        }
    std::vector<double> lam, V;
    std::vector<char> kept;
    pinv_spectrum(A, K, rtol, lam, V, kept);
    pinv_directional(lam, V, kept, K, dA.data(), M);
}

void centers_gradient(const float* centers, int K, int rho, double sigma_r, double rtol, const double* Gm,
                      const double* S1, const double* S2, double* grad) {
    std::fill(grad, grad + (size_t)K * rho, 0.0);
    if (std::isinf(sigma_r)) return;  // b = 1 and A = 1: nothing depends on the centers
    const double is2 = 1.0 / (sigma_r * sigma_r);
    // through b_l(i): sum_i w_l(i) (p(i) - mu_l) / sigma_r^2
    for (int k = 0; k < K; ++k)
        for (int t = 0; t < rho; ++t)
            grad[(size_t)k * rho + t] = (S2[(size_t)k * rho + t] - S1[k] * (double)centers[(size_t)k * rho + t]) * is2;
    // through A: dL/dA = the pseudo-inverse derivative map applied to
    // dL/dA^+ = Gm (symmetrised: A is symmetric), then
    // dA_kl / dmu_k = A_kl (mu_l - mu_k) / sigma_r^2 for l != k
    std::vector<double> A((size_t)K * K), Gs((size_t)K * K), GA((size_t)K * K);
    kernel_matrix(centers, K, rho, sigma_r, A.data());
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) Gs[(size_t)k * K + l] = 0.5 * (Gm[(size_t)k * K + l] + Gm[(size_t)l * K + k]);
    std::vector<double> lam, V;
    std::vector<char> kept;
    pinv_spectrum(A, K, rtol, lam, V, kept);
    pinv_directional(lam, V, kept, K, Gs.data(), GA.data());
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) {
            if (l == k) continue;
            const double c = 2.0 * GA[(size_t)k * K + l] * A[(size_t)k * K + l] * is2;  // A_kl and A_lk
            for (int t = 0; t < rho; ++t)
                grad[(size_t)k * rho + t] +=
                    c * ((double)centers[(size_t)l * rho + t] - (double)centers[(size_t)k * rho + t]);
        }
}

}  // namespace fhd
