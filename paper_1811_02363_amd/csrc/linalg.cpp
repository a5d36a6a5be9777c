// The K x K least-squares solve of Algorithm 1 (eqs. (11)-(12)): the kernel
// matrix A_kl = phi(mu_k - mu_l) and its Moore-Penrose pseudo-inverse, in FP64
// on the host.  A is symmetric, so its singular values are |eigenvalues| and
// A^+ = sum over kept eigenpairs of v v^T / lambda.  The eigen-decomposition
// is the cyclic Jacobi method (rotations zeroing one off-diagonal pair at a
// time, swept until the off-diagonal mass is negligible).
#include <algorithm>
#include <cmath>
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

namespace {

// Eigen-decomposition of the symmetric K x K matrix `a` (destroyed): on return
// lam[i] are the eigenvalues and column i of v (row-major K x K) the
// corresponding unit eigenvector.
void jacobi_eigen(std::vector<double>& a, int K, std::vector<double>& lam, std::vector<double>& v) {
    v.assign((size_t)K * K, 0.0);
    for (int i = 0; i < K; ++i) v[(size_t)i * K + i] = 1.0;
    double fro = 0.0;
    for (double x : a) fro += x * x;
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < K; ++p)
            for (int q = p + 1; q < K; ++q) off += a[(size_t)p * K + q] * a[(size_t)p * K + q];
        if (std::sqrt(2.0 * off) <= 1e-16 * fro || off == 0.0) break;
        for (int p = 0; p < K - 1; ++p) {
            for (int q = p + 1; q < K; ++q) {
                const double apq = a[(size_t)p * K + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * K + p], aqq = a[(size_t)q * K + q];
                // rotation angle that zeroes a_pq: tan(theta) = t
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // a <- J^T a J, J = identity but J_pp = J_qq = c, J_pq = s, J_qp = -s
                for (int k = 0; k < K; ++k) {
                    const double akp = a[(size_t)k * K + p], akq = a[(size_t)k * K + q];
                    a[(size_t)k * K + p] = c * akp - s * akq;
                    a[(size_t)k * K + q] = s * akp + c * akq;
                }
                for (int k = 0; k < K; ++k) {
                    const double apk = a[(size_t)p * K + k], aqk = a[(size_t)q * K + k];
                    a[(size_t)p * K + k] = c * apk - s * aqk;
                    a[(size_t)q * K + k] = s * apk + c * aqk;
                }
                a[(size_t)p * K + q] = 0.0;
                a[(size_t)q * K + p] = 0.0;
                for (int k = 0; k < K; ++k) {
                    const double vkp = v[(size_t)k * K + p], vkq = v[(size_t)k * K + q];
                    v[(size_t)k * K + p] = c * vkp - s * vkq;
                    v[(size_t)k * K + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    lam.resize(K);
    for (int i = 0; i < K; ++i) lam[i] = a[(size_t)i * K + i];
}

}  // namespace

PinvResult pinv_symmetric(const double* A, int K, double rtol, double* P) {
    std::vector<double> a(A, A + (size_t)K * K), lam, v;
    jacobi_eigen(a, K, lam, v);
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

}  // namespace fhd
