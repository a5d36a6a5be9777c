// The guide of nonlocal means (Sec. I-A, Sec. III-C): every pixel's m x m x n
// patch, projected onto the leading principal directions of all patches.
//
//   moments pass:  per block of pixels, sums of x and of x x^T (upper
//                  triangle) over the block's patches (x = patch - 1/2),
//                  FP32 within 256-pixel runs, FP64 across runs; on the
//                  matrix cores for patches of up to 95 coordinates;
//   reduce pass:   the blocks' sums added in a fixed order (FP64): runs of
//                  blocks, then the runs in order;
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

typedef float f32x16 __attribute__((ext_vector_type(16)));

// The moments on the matrix cores (patches of at most MC_D = 95 coordinates).
// A wave takes 256 of the block's pixels (four tile rows of 64).  Its patch
// vectors, with a constant 1 appended (whose products give the first
// moments) and zeros up to 96, form X^T X as the six upper-triangle 32 x 32
// tiles of a 96 x 96 product: 128 steps of v_mfma_f32_32x32x2f32 per tile,
// two pixels a step, the six tiles' products independent (so their latency
// overlaps).  Lane l supplies coordinate 32 b + l % 32 of pixel 2 s + l / 32
// for each row block b, which is the A operand of tiles (b, .) and the B
// operand of tiles (., b); it receives C[i][l % 32] for the rows
// i = 8 (r / 4) + 4 (l / 32) + r % 4.  FP32 over the wave's 256 pixels (the
// runs of the vector form), FP64 across the four waves in order.
constexpr int MC_D = 95;

__global__ __launch_bounds__(NT) void pca_moments_mfma(const float* __restrict__ f, int n, int H, int W, int m,
                                                       int gx, double* __restrict__ part) {
    extern __shared__ float lds[];
    const int D = m * m * n;
    const int E = D + D * (D + 1) / 2;
    const int by = (blockIdx.x / gx) * TPY, bx = (blockIdx.x % gx) * TPX;
    const int tx = TPX + m - 1;
    float* tile = lds;
    double* rec = reinterpret_cast<double*>(lds + ((n * (TPY + m - 1) * tx + 1) & ~1));
    stage_tile(f, n, H, W, m, by, bx, 0.5f, tile);
    __syncthreads();
    const int ny = min(TPY, H - by), nx = min(TPX, W - bx);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, jr = lane & 31, kh = lane >> 5;
    int off[3], kind[3];  // kind: 0 a patch coordinate, 1 the constant 1, 2 padding
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int j = 32 * b + jr;
        kind[b] = j < D ? 0 : (j == D ? 1 : 2);
        off[b] = j < D ? coord_off(j, n, m) : 0;
    }
    f32x16 acc[6];
#pragma unroll
    for (int t = 0; t < 6; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
    for (int s = 0; s < 128; ++s) {
        const int p = 2 * s + kh;  // pixel of the wave's 256
        const int py = 4 * wave + (p >> 6), px = p & 63;
        const bool in = py < ny && px < nx;
        const int po = py * tx + px;
        float v[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) v[b] = !in ? 0.0f : (kind[b] == 0 ? tile[off[b] + po] : (kind[b] == 1 ? 1.0f : 0.0f));
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[0], v[0], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[0], v[1], acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[0], v[2], acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[1], v[1], acc[3], 0, 0, 0);
        acc[4] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[1], v[2], acc[4], 0, 0, 0);
        acc[5] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[2], v[2], acc[5], 0, 0, 0);
    }
    // record entry e = J (first moment, K = the constant) or D + (row start
    // of J) + K - J for J <= K < D; the waves add in order
    // (one tile at a time, picked by a uniform switch, so only its sixteen
    // values and entries are live)
    for (int w = 0; w < NT / 64; ++w) {
        if (wave == w) {
#pragma unroll 1
            for (int t = 0; t < 6; ++t) {
                f32x16 cur;
                switch (t) {
                    case 0: cur = acc[0]; break;
                    case 1: cur = acc[1]; break;
                    case 2: cur = acc[2]; break;
                    case 3: cur = acc[3]; break;
                    case 4: cur = acc[4]; break;
                    default: cur = acc[5]; break;
                }
                const int tr = t < 3 ? 0 : (t < 5 ? 1 : 2), tc = t < 3 ? t : (t < 5 ? t - 2 : 2);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int J = 32 * tr + 8 * (r >> 2) + 4 * kh + (r & 3), K = 32 * tc + jr;
                    int e = -1;
                    if (K == D && J < D) e = J;
                    else if (J <= K && K < D) e = D + J * D - J * (J - 1) / 2 + (K - J);
                    if (e >= 0) rec[e] = (w == 0 ? 0.0 : rec[e]) + (double)cur[r];
                }
            }
        }
        __syncthreads();
    }
    double* out = part + (long long)blockIdx.x * E;
    for (int e = threadIdx.x; e < E; e += NT) out[e] = rec[e];
}

// Block sums in a fixed order: chunk c adds blocks c, c + C, c + 2C, ... of
// entry e; pca_reduce_chunks adds the C chunks in order.
constexpr int RC = 32;

__global__ __launch_bounds__(NT) void pca_reduce(const double* __restrict__ part, int nb, int E,
                                                 double* __restrict__ chunk) {
    const int e = blockIdx.x * NT + threadIdx.x, c = blockIdx.y;
    if (e >= E) return;
    double s = 0.0;
    for (int b = c; b < nb; b += RC) s += part[(long long)b * E + e];
    chunk[(long long)c * E + e] = s;
}

__global__ __launch_bounds__(NT) void pca_reduce_chunks(const double* __restrict__ chunk, int E,
                                                        double* __restrict__ out) {
    const int e = blockIdx.x * NT + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int c = 0; c < RC; ++c) s += chunk[(long long)c * E + e];
    out[e] = s;
}

// guide[d][pixel] = sum_j (x_j - mean_j) V[j][d]; V and mean in `pv`
// (D x dims, then D), staged in LDS after the tile, with the tile offset of
// every patch coordinate.  A thread takes four adjacent pixels of a tile row
// (the tile's 16 x 64 pixels are one pass of the 256 threads), so each read
// of a row of V serves four outputs.
constexpr int PX4 = 4;
static_assert(TPY * TPX == NT * PX4, "one pass of four pixels per thread");

__global__ __launch_bounds__(NT) void pca_project(const float* __restrict__ f, int n, int H, int W, int m,
                                                  int gx, int dims, const float* __restrict__ pv,
                                                  float* __restrict__ guide) {
    extern __shared__ float lds[];
    const int D = m * m * n;
    const int ty = TPY + m - 1, tx = TPX + m - 1;
    float* tile = lds;
    float* sv = tile + n * ty * tx;
    float* smean = sv + D * dims;
    int* soff = reinterpret_cast<int*>(smean + D);  // tile offset of each patch coordinate
    const int by = (blockIdx.x / gx) * TPY, bx = (blockIdx.x % gx) * TPX;
    stage_tile(f, n, H, W, m, by, bx, 0.0f, tile);
    for (int e = threadIdx.x; e < D * dims + D; e += NT) sv[e] = pv[e];
    for (int j = threadIdx.x; j < D; j += NT) soff[j] = coord_off(j, n, m);
    __syncthreads();
    const int py = threadIdx.x / (TPX / PX4), px0 = (threadIdx.x % (TPX / PX4)) * PX4;
    const int y = by + py;
    const long long HW = (long long)H * W;
    for (int d0 = 0; d0 < dims; d0 += 16) {
        float acc[PX4][16];
#pragma unroll
        for (int u = 0; u < PX4; ++u)
#pragma unroll
            for (int t = 0; t < 16; ++t) acc[u][t] = 0.0f;
        for (int j = 0; j < D; ++j) {
            const float* tp = tile + soff[j] + py * tx + px0;
            const float mj = smean[j];
            float xj[PX4];
#pragma unroll
            for (int u = 0; u < PX4; ++u) xj[u] = tp[u] - mj;
            const float* vr = sv + j * dims + d0;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const float vt = d0 + t < dims ? vr[t] : 0.0f;
#pragma unroll
                for (int u = 0; u < PX4; ++u) acc[u][t] = fmaf(xj[u], vt, acc[u][t]);
            }
        }
        if (y < H) {
#pragma unroll
            for (int u = 0; u < PX4; ++u) {
                const int x = bx + px0 + u;
                if (x >= W) break;
#pragma unroll
                for (int t = 0; t < 16; ++t)
                    if (d0 + t < dims) guide[(d0 + t) * HW + (long long)y * W + x] = acc[u][t];
            }
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
    probe.take<double>((size_t)RC * E);
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
    double* chunk = ws.take<double>((size_t)RC * E);
    double* sums = ws.take<double>((size_t)E);
    float* pv = ws.take<float>((size_t)D * dims + D);
    hipStream_t st = c.stream;
    const size_t tile_bytes = sizeof(float) * n * (TPY + m - 1) * (TPX + m - 1);
    if (D <= MC_D) {
        const size_t lds = sizeof(float) * (((size_t)n * (TPY + m - 1) * (TPX + m - 1) + 1) & ~(size_t)1) +
                           sizeof(double) * E;
        FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(pca_moments_mfma),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(pca_moments_mfma, dim3(nb), dim3(NT), lds, st, f, n, H, W, m, gx, part);
    } else {
        hipLaunchKernelGGL(pca_moments, dim3(nb), dim3(NT), tile_bytes, st, f, n, H, W, m, gx, part);
    }
    hipLaunchKernelGGL(pca_reduce, dim3((E + NT - 1) / NT, RC), dim3(NT), 0, st, part, nb, E, chunk);
    hipLaunchKernelGGL(pca_reduce_chunks, dim3((E + NT - 1) / NT), dim3(NT), 0, st, chunk, E, sums);
    FHD_HIP(hipGetLastError());
    // the sums come back through pinned memory (a direct copy, no staging)
    double* pin = static_cast<double*>(c.host_stage(1, sizeof(double) * E));
    FHD_HIP(hipMemcpyAsync(pin, sums, sizeof(double) * E, hipMemcpyDeviceToHost, st));
    FHD_HIP(hipStreamSynchronize(st));
    std::vector<double> hs(pin, pin + E);
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
    const size_t lds = tile_bytes + sizeof(float) * ((size_t)D * dims + D) + sizeof(int) * D;
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(pca_project),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(pca_project, dim3(nb), dim3(NT), lds, st, f, n, H, W, m, gx, dims, pv, guide);
    FHD_HIP(hipGetLastError());
}

}  // namespace fhd
