// Eq. (10) solved at every pixel (Sec. II-A): the coefficients c*(i) of the
// least-squares fit of phi(x - p(i)) by the K basis functions phi(x - mu_k)
// over the window's own guide samples x in Theta_i, the guide values of the
// in-image pixels q_1 .. q_m of the (2S+1)^2 window around i.  With the
// m x K design matrix M_i of rows b(q_j) (the weights of eq. (12) at q_j) and
// the targets y_j = phi(p(q_j) - p(i)), c*(i) = M_i^+ y_i is the minimum-norm
// minimiser.  The paper uses it to judge its surrogate eq. (11), whose
// solution c = A^+ b(i) shares one pseudo-inverse across all pixels.
//
// One wave per pixel, FP64 throughout (inputs are the FP32 guide and
// centers, outputs FP32):
//  1. the rows [b(q_j), y_j] are formed 64 at a time, one per lane, into LDS;
//  2. a streaming Givens QR folds each row into the upper triangle R of
//     [M | y]: lane c holds column c, and rotation k takes its pivot R[k][k]
//     and the row's entry k from lane k.  The solve therefore sees the
//     singular values of M itself, not those of the squared normal matrix.
//     Column K gives z = Q^T y, and the part of each row left after the K
//     rotations adds up to rho^2, the residual of the full-rank fit;
//  3. a one-sided Jacobi SVD of the K x K triangle (Hestenes: column pairs in
//     a round-robin order, lane c holds column c of R V and of V, the pair
//     exchanging columns through LDS) gives R V = U Sigma; singular values at
//     or below max(m, K) 2^-52 sigma_max are dropped, the tolerance of the
//     pseudo-inverse A^+ of the filter (the MATLAB default);
//  4. c* = sum over the kept c of v_c (u_c . z) / sigma_c.  The minimum of
//     eq. (10) is rho^2 + |z - R c*|^2, and eq. (10) at the surrogate's
//     c = A^+ b(i) is rho^2 + |z - R c|^2 likewise.
#include <cmath>

#include "fhd_internal.h"

namespace fhd {
namespace {

constexpr int EL_T = 64;  // threads per block: one wave, one pixel

struct ELArgs {
    const float* guide;  // rho planes of N pixels
    const float* mu;     // K x rho centers
    const double* P;     // K x K A^+ (row-major), or null
    float* coef;         // K planes (plane stride cstride, row pitch cpitch), or null
    float* obj;          // N: the minimum of eq. (10), or null
    float* obj11;        // N: eq. (10) at c = A^+ b(i), or null (needs P)
    long long N, cstride;
    int rho, H, W, S, K, cpitch;
    double inv2s2;       // 1 / (2 sigma_r^2), 0 for sigma_r = inf
};

// the value of v in lane `lane` (uniform)
__device__ __forceinline__ double lane_value(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Round-robin pairing of KP (even) columns, column 0 fixed: the partner of
// column c in round r (every pair meets once in KP - 1 rounds).
__device__ __forceinline__ int rr_partner(int c, int r, int KP) {
    const int L = KP - 1;
    const int pos = c == 0 ? 0 : (((c - 1 - r) % L) + L) % L + 1;
    const int pp = KP - 1 - pos;
    return pp == 0 ? 0 : (pp - 1 + r) % L + 1;
}

template <int KM>
__global__ __launch_bounds__(EL_T) void exact_ls_kernel(ELArgs a) {
    extern __shared__ double sh[];
    double* rows = sh;                          // EL_T x (KM + 1): the batch's rows [b(q_j), y_j]
    double* colv = rows + EL_T * (KM + 1);      // KM x KM: column c of R V at c KM
    double* vcol = colv + KM * KM;              // KM x KM: column c of V at c KM
    double* Rs = vcol + KM * KM;                // KM x (KM + 1): R and z, entry (k, c) at k (KM + 1) + c
    double* vec = Rs + KM * (KM + 1);           // 3 KM: b(i), c*, A^+ b(i)
    const int K = a.K, lane = threadIdx.x;
    const long long i = blockIdx.x;
    const int iy = (int)(i / a.W), ix = (int)(i - (long long)iy * a.W);
    const int y0 = max(0, iy - a.S), y1 = min(a.H - 1, iy + a.S);
    const int x0 = max(0, ix - a.S), x1 = min(a.W - 1, ix + a.S);
    const int wx = x1 - x0 + 1, m = (y1 - y0 + 1) * wx;

    // 1-2: streaming QR of [M | y]
    double R[KM];  // lane c: R[k][c] for k < K (upper triangle; lane K: z_k)
#pragma unroll
    for (int k = 0; k < KM; ++k) R[k] = 0.0;
    double rho2 = 0.0;  // lane K: the residual of the full-rank fit, squared
    for (int base = 0; base < m; base += EL_T) {
        const int nb = min(EL_T, m - base);
        if (lane < nb) {
            const int j = base + lane;
            const int qy = y0 + j / wx, qx = x0 + j % wx;
            const long long q = (long long)qy * a.W + qx;
            double* row = rows + lane * (KM + 1);
            double d2 = 0.0;
            for (int r = 0; r < a.rho; ++r) {
                const double d = (double)a.guide[r * a.N + q] - (double)a.guide[r * a.N + i];
                d2 = fma(d, d, d2);
            }
            row[K] = exp(-d2 * a.inv2s2);
            for (int k = 0; k < K; ++k) {
                double e2 = 0.0;
                for (int r = 0; r < a.rho; ++r) {
                    const double d = (double)a.guide[r * a.N + q] - (double)a.mu[k * a.rho + r];
                    e2 = fma(d, d, e2);
                }
                row[k] = exp(-e2 * a.inv2s2);
            }
        }
        __syncthreads();
        for (int j = 0; j < nb; ++j) {
            double w = lane <= K ? rows[j * (KM + 1) + lane] : 0.0;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (k < K) {  // uniform
                    const double piv = lane_value(R[k], k), b = lane_value(w, k);
                    if (b != 0.0) {  // uniform
                        const double s2 = fma(piv, piv, b * b);
                        const double inv = rsqrt(s2);
                        const double cs = piv * inv, sn = b * inv;
                        if (lane > k) {
                            const double t = R[k];
                            R[k] = fma(cs, t, sn * w);
                            w = fma(cs, w, -sn * t);
                        } else if (lane == k) {
                            R[k] = s2 * inv;
                            w = 0.0;
                        }
                    }
                }
            }
            if (lane == K) rho2 = fma(w, w, rho2);
        }
        __syncthreads();
    }
    const double res2 = lane_value(rho2, K);
    if (lane <= K) {
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < K) Rs[k * (KM + 1) + lane] = R[k];
    }

    // 3: one-sided Jacobi SVD of the K x K triangle
    const int KP = K + (K & 1);
    double v[KM];
    const bool mine = lane < K;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (!mine) R[k] = 0.0;
        v[k] = (mine && k == lane) ? 1.0 : 0.0;
    }
    if (lane < KP) {
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            colv[lane * KM + k] = R[k];
            vcol[lane * KM + k] = v[k];
        }
    }
    __syncthreads();
    constexpr double EPS = 2.220446049250313e-16;  // 2^-52
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int r = 0; r < KP - 1; ++r) {
            const int q = lane < KP ? rr_partner(lane, r, KP) : lane;
            const double* oc = colv + q * KM;
            double own2 = 0.0, oth2 = 0.0, g = 0.0;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (k < K) {
                    const double o = oc[k];
                    own2 = fma(R[k], R[k], own2);
                    oth2 = fma(o, o, oth2);
                    g = fma(R[k], o, g);
                }
            }
            // both lanes of a pair form the same rotation from the same sums
            const bool lo = lane < q;
            const double alo = lo ? own2 : oth2, ahi = lo ? oth2 : own2;
            const bool rot = lane < KP && q != lane && g != 0.0 && fabs(g) > EPS * sqrt(alo) * sqrt(ahi);
            if (rot) {
                const double zeta = (ahi - alo) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
                const double cs = rsqrt(fma(t, t, 1.0)), sn = cs * t;
                const double* ov = vcol + q * KM;
#pragma unroll
                for (int k = 0; k < KM; ++k) {
                    if (k < K) {
                        const double o = oc[k], ovk = ov[k];
                        R[k] = lo ? fma(cs, R[k], -sn * o) : fma(sn, o, cs * R[k]);
                        v[k] = lo ? fma(cs, v[k], -sn * ovk) : fma(sn, ovk, cs * v[k]);
                    }
                }
                rotated = 1;
            }
            __syncthreads();  // every partner column read
            if (rot) {
#pragma unroll
                for (int k = 0; k < KM; ++k) {
                    if (k < K) {
                        colv[lane * KM + k] = R[k];
                        vcol[lane * KM + k] = v[k];
                    }
                }
            }
            __syncthreads();
        }
        if (!__any(rotated)) break;
    }

    // 4: c* = sum over the kept singular triplets of v_c (u_c . z) / sigma_c
    double s2 = 0.0, dz = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < K) {
            s2 = fma(R[k], R[k], s2);
            dz = fma(R[k], Rs[k * (KM + 1) + K], dz);
        }
    }
    const double sig = mine ? sqrt(s2) : 0.0;
    const double tol = (double)max(m, K) * EPS * wave_max(sig);
    const double wgt = (mine && sig > tol) ? dz / s2 : 0.0;
    __syncthreads();
    if (mine) {
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < K) colv[lane * KM + k] = wgt * v[k];
        // b(i), for eq. (10) at the surrogate's coefficients
        double e2 = 0.0;
        for (int r = 0; r < a.rho; ++r) {
            const double d = (double)a.guide[r * a.N + i] - (double)a.mu[lane * a.rho + r];
            e2 = fma(d, d, e2);
        }
        vec[lane] = exp(-e2 * a.inv2s2);
    }
    __syncthreads();
    double cstar = 0.0;
    if (mine) {
        for (int c = 0; c < K; ++c) cstar += colv[c * KM + lane];
        vec[KM + lane] = cstar;
        if (a.P != nullptr) {
            double c11 = 0.0;
            for (int l = 0; l < K; ++l) c11 = fma(a.P[lane * K + l], vec[l], c11);
            vec[2 * KM + lane] = c11;
        }
    }
    __syncthreads();
    // the residual z - R c (R upper triangular), for c* and for A^+ b(i)
    double r1 = 0.0, r2 = 0.0;
    if (mine) {
        double rc = 0.0, rc11 = 0.0;
        for (int c = lane; c < K; ++c) {
            rc = fma(Rs[lane * (KM + 1) + c], vec[KM + c], rc);
            if (a.P != nullptr) rc11 = fma(Rs[lane * (KM + 1) + c], vec[2 * KM + c], rc11);
        }
        r1 = Rs[lane * (KM + 1) + K] - rc;
        r2 = Rs[lane * (KM + 1) + K] - rc11;
    }
    const double o10 = res2 + wave_sum(r1 * r1);
    const double o11 = res2 + wave_sum(r2 * r2);
    if (mine && a.coef != nullptr) a.coef[lane * a.cstride + (long long)iy * a.cpitch + ix] = (float)cstar;
    if (lane == 0) {
        if (a.obj != nullptr) a.obj[i] = (float)o10;
        if (a.obj11 != nullptr) a.obj11[i] = (float)o11;
    }
}

template <int KM>
size_t exact_ls_lds() {
    return sizeof(double) * ((size_t)EL_T * (KM + 1) + 2 * KM * KM + (size_t)KM * (KM + 1) + 3 * KM);
}

}  // namespace

void exact_ls_run(Ctx& c, const float* guide, int rho, int H, int W, const float* mu_dev, int K,
                  const double* P_dev, double sigma_r, int S, float* coef, long long cstride, int cpitch, float* obj,
                  float* obj11) {
    FHD_REQUIRE(K >= 1 && K <= EXACT_LS_MAX_K, FHD_EUNSUPPORTED, "the per-pixel least squares supports K <= 32");
    FHD_REQUIRE(obj11 == nullptr || P_dev != nullptr, FHD_EINVAL, "internal: eq. (10) at A^+ b needs A^+");
    ELArgs a;
    a.guide = guide;
    a.mu = mu_dev;
    a.P = P_dev;
    a.coef = coef;
    a.obj = obj;
    a.obj11 = obj11;
    a.N = (long long)H * W;
    a.cstride = cstride;
    a.rho = rho;
    a.H = H;
    a.W = W;
    a.S = S;
    a.K = K;
    a.cpitch = cpitch;
    a.inv2s2 = std::isinf(sigma_r) ? 0.0 : 1.0 / (2.0 * sigma_r * sigma_r);
    FHD_REQUIRE(a.N < (1LL << 31), FHD_EUNSUPPORTED, "image has 2^31 pixels or more");
    const dim3 g((unsigned)a.N);
    hipEvent_t t0 = c.stage_begin();
    if (K <= 8) {
        hipLaunchKernelGGL(exact_ls_kernel<8>, g, dim3(EL_T), exact_ls_lds<8>(), c.stream, a);
    } else if (K <= 16) {
        hipLaunchKernelGGL(exact_ls_kernel<16>, g, dim3(EL_T), exact_ls_lds<16>(), c.stream, a);
    } else {
        const size_t lds = exact_ls_lds<32>();
        FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(exact_ls_kernel<32>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(exact_ls_kernel<32>, g, dim3(EL_T), lds, c.stream, a);
    }
    c.stage_end(FHD_STAGE_WEIGHTS, t0);
    FHD_HIP(hipGetLastError());
}

}  // namespace fhd
