// The guide of nonlocal means (Sec. I-A, Sec. III-C): every pixel's m x m x n
// patch, projected onto the leading principal directions of all patches.
//
//   moments pass:  per block of pixels, sums of x and of x x^T (upper
//                  triangle) over the block's patches (x = patch - 1/2),
//                  FP32 within 256-pixel runs, FP64 across runs;
//   reduce pass:   the blocks' sums added in block order (FP64);
//   host:          covariance (FP64), symmetric eigen-decomposition, the
//                  `dims` leading eigenvectors (sign: largest-magnitude
//                  component positive);
//   projection:    guide_d(i) = sum_j (x_j(i) - mean_j) V_jd.
// Patches are flattened in (dy, dx, channel) order; the image is extended by
// half-sample symmetric reflection (index -1 reads 0).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "fhd_internal.h"

namespace fhd {
namespace {

constexpr int NT = 256;
constexpr int TPY = 16, TPX = 64;  // pixels per block tile
constexpr int MAXD = 160;          // patch dimension limit (m*m*n)

__device__ __forceinline__ int reflect(int i, int L) {
    while (i < 0 || i >= L) i = i < 0 ? -i - 1 : 2 * L - i - 1;
    return i;
}

// stage the tile's image values (minus `shift`) with an (m-1)-pixel apron
__device__ void stage_tile(const float* f, int n, int H, int W, int m, int by, int bx, float shift, float* t) {
    const int h = m / 2;
    const int ty = TPY + m - 1, tx = TPX + m - 1;
    for (int e = threadIdx.x; e < n * ty * tx; e += NT) {
        const int c = e / (ty * tx), r = e - c * ty * tx;
        const int yy = reflect(by - h + r / tx, H), xx = reflect(bx - h + r % tx, W);
        t[e] = f[(long long)c * H * W + (long long)yy * W + xx] - shift;
    }
}

// offset of patch coordinate j inside the staged tile, for the tile's pixel (0,0)
__device__ __forceinline__ int coord_off(int j, int n, int m) {
    const int c = j % n, dx = (j / n) % m, dy = j / (n * m);
    return c * (TPY + m - 1) * (TPX + m - 1) + dy * (TPX + m - 1) + dx;
}

__global__ __launch_bounds__(NT) void pca_moments(const float* __restrict__ f, int n, int H, int W, int m,
                                                  int gx, double* __restrict__ part) {
    extern __shared__ float tile[];
    const int D = m * m * n;
    const int E = D + D * (D + 1) / 2;
    const int by = (blockIdx.x / gx) * TPY, bx = (blockIdx.x % gx) * TPX;
    stage_tile(f, n, H, W, m, by, bx, 0.5f, tile);
    __syncthreads();
    const int tx = TPX + m - 1;
    const int ny = min(TPY, H - by), nx = min(TPX, W - bx);
    double* out = part + (long long)blockIdx.x * E;
    for (int e = threadIdx.x; e < E; e += NT) {
        int j, k;
        if (e < D) {
            j = e;
            k = -1;
        } else {
            // e - D enumerates the pairs j <= k row by row
            int r = e - D;
            j = 0;
            while (r >= D - j) {
                r -= D - j;
                ++j;
            }
            k = j + r;
        }
        const int oj = coord_off(j, n, m), ok = k >= 0 ? coord_off(k, n, m) : 0;
        double tot = 0.0;
        float run = 0.0f;
        int cnt = 0;
        for (int py = 0; py < ny; ++py) {
            for (int px = 0; px < nx; ++px) {
                const int p = py * tx + px;
                const float xj = tile[oj + p];
                run = k >= 0 ? fmaf(xj, tile[ok + p], run) : run + xj;
                if (++cnt == 256) {
                    tot += run;
                    run = 0.0f;
                    cnt = 0;
                }
            }
        }
        out[e] = tot + run;
    }
}

__global__ __launch_bounds__(NT) void pca_reduce(const double* __restrict__ part, int nb, int E,
                                                 double* __restrict__ out) {
    const int e = blockIdx.x * NT + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(long long)b * E + e];
    out[e] = s;
}

// guide[d][pixel] = sum_j (x_j - mean_j) V[j][d]; V and mean in `pv`
// (D x dims, then D), staged in LDS after the tile.
__global__ __launch_bounds__(NT) void pca_project(const float* __restrict__ f, int n, int H, int W, int m,
                                                  int gx, int dims, const float* __restrict__ pv,
                                                  float* __restrict__ guide) {
    extern __shared__ float lds[];
    const int D = m * m * n;
    const int ty = TPY + m - 1, tx = TPX + m - 1;
    float* tile = lds;
    float* sv = tile + n * ty * tx;
    float* smean = sv + D * dims;
    const int by = (blockIdx.x / gx) * TPY, bx = (blockIdx.x % gx) * TPX;
    stage_tile(f, n, H, W, m, by, bx, 0.0f, tile);
    for (int e = threadIdx.x; e < D * dims + D; e += NT) sv[e] = pv[e];
    __syncthreads();
    for (int q = threadIdx.x; q < TPY * TPX; q += NT) {
        const int py = q / TPX, px = q % TPX;
        const int y = by + py, x = bx + px;
        if (y >= H || x >= W) continue;
        float acc[16];
        for (int d0 = 0; d0 < dims; d0 += 16) {
#pragma unroll
            for (int t = 0; t < 16; ++t) acc[t] = 0.0f;
            for (int j = 0; j < D; ++j) {
                const float xj = tile[coord_off(j, n, m) + py * tx + px] - smean[j];
                const float* vr = sv + j * dims + d0;
#pragma unroll
                for (int t = 0; t < 16; ++t)
                    if (d0 + t < dims) acc[t] = fmaf(xj, vr[t], acc[t]);
            }
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (d0 + t < dims) guide[(long long)(d0 + t) * H * W + (long long)y * W + x] = acc[t];
        }
    }
}

}  // namespace

size_t nlm_workspace(int n, int H, int W, int m, int dims) {
    const int D = m * m * n;
    const int E = D + D * (D + 1) / 2;
    const long long nb = (long long)((H + TPY - 1) / TPY) * ((W + TPX - 1) / TPX);
    Arena probe;
    probe.take<double>((size_t)nb * E);
    probe.take<double>((size_t)E);
    probe.take<float>((size_t)D * dims + D);
    return probe.used;
}

void nlm_guide_run(Ctx& c, Arena& ws, const float* f, int n, int H, int W, int m, int dims, float* guide,
                   double* eigvals) {
    const int D = m * m * n;
    FHD_REQUIRE(m >= 1 && (m & 1) == 1, FHD_EINVAL, "patch size must be odd");
    FHD_REQUIRE(D <= MAXD, FHD_EUNSUPPORTED, "patch dimension m*m*n exceeds 160");
    FHD_REQUIRE(dims >= 1 && dims <= D && dims <= FHD_MAX_RHO, FHD_EINVAL, "dims must be in [1, min(m*m*n, 64)]");
    const int E = D + D * (D + 1) / 2;
    const int gx = (W + TPX - 1) / TPX, gy = (H + TPY - 1) / TPY;
    const int nb = gx * gy;
    double* part = ws.take<double>((size_t)nb * E);
    double* sums = ws.take<double>((size_t)E);
    float* pv = ws.take<float>((size_t)D * dims + D);
    hipStream_t st = c.stream;
    const size_t tile_bytes = sizeof(float) * n * (TPY + m - 1) * (TPX + m - 1);
    hipLaunchKernelGGL(pca_moments, dim3(nb), dim3(NT), tile_bytes, st, f, n, H, W, m, gx, part);
    hipLaunchKernelGGL(pca_reduce, dim3((E + NT - 1) / NT), dim3(NT), 0, st, part, nb, E, sums);
    FHD_HIP(hipGetLastError());
    std::vector<double> hs(E);
    FHD_HIP(hipMemcpyAsync(hs.data(), sums, sizeof(double) * E, hipMemcpyDeviceToHost, st));
    FHD_HIP(hipStreamSynchronize(st));
    const double N = (double)H * W;
    std::vector<double> mean(D), cov((size_t)D * D);
    for (int j = 0; j < D; ++j) mean[j] = hs[j] / N;
    {
        int e = D;
        for (int j = 0; j < D; ++j)
            for (int k = j; k < D; ++k, ++e) {
                const double v = hs[e] / N - mean[j] * mean[k];
                cov[(size_t)j * D + k] = cov[(size_t)k * D + j] = v;
            }
    }
    std::vector<double> lam, V;
    sym_eigen_checked(cov, D, lam, V, "the patch covariance");
    std::vector<int> order(D);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
    if (eigvals)
        for (int i = 0; i < D; ++i) eigvals[i] = lam[order[i]];
    std::vector<float> hv((size_t)D * dims + D);
    for (int d = 0; d < dims; ++d) {
        const int col = order[d];
        int big = 0;
        for (int j = 1; j < D; ++j)
            if (std::fabs(V[(size_t)j * D + col]) > std::fabs(V[(size_t)big * D + col])) big = j;
        const double sgn = V[(size_t)big * D + col] < 0.0 ? -1.0 : 1.0;
        for (int j = 0; j < D; ++j) hv[(size_t)j * dims + d] = (float)(sgn * V[(size_t)j * D + col]);
    }
    for (int j = 0; j < D; ++j) hv[(size_t)D * dims + j] = (float)(mean[j] + 0.5);
    char* stage = static_cast<char*>(c.host_stage(2, sizeof(float) * hv.size()));
    std::memcpy(stage, hv.data(), sizeof(float) * hv.size());
    FHD_HIP(hipMemcpyAsync(pv, stage, sizeof(float) * hv.size(), hipMemcpyHostToDevice, st));
    c.stage_done(2);
    const size_t lds = tile_bytes + sizeof(float) * ((size_t)D * dims + D);
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(pca_project),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(pca_project, dim3(nb), dim3(NT), lds, st, f, n, H, W, m, gx, dims, pv, guide);
    FHD_HIP(hipGetLastError());
}

}  // namespace fhd
