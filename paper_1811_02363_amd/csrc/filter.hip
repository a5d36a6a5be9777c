// Steps 3-5 of Algorithm 1 (Sec. II-B) on gfx950: range weights and
// coefficients, the (n+1)K spatial convolutions of eqs. (13)-(14) and the
// recombination of eqs. (15)-(16), plus the brute-force filter of
// eqs. (1)-(2).
//
// The convolutions run as two passes over (n+1)K FP32 planes:
//   row pass:    for every cluster l, U_l = g_l * [f, 1] is formed on the fly
//                from the guide and filtered along x (LDS-staged halo row);
//                the K(n+1) row-filtered planes are written once;
//   column pass: reads them once, filters along y, and recombines per pixel
//                with weight h_l(i), writing g_hat and the normaliser.
// For least-squares coefficients c = A^+ b the pair (g, h) is (c, b): since
// A^+ is symmetric, sum_k c_k(i) b_k(i-j) = sum_l b_l(i) c_l(i-j), so the
// recombination of eqs. (15)-(16) equals sum_l b_l(i) (w * c_l [f,1])(i) and
// only the cheap b_l(i) is needed where the output is formed.  For the hard
// assignment of eq. (17) the pair is (b, 1[s(i) = l]) (the form of Alg. 1).
// The Gaussian window is separable and zero extension commutes with the row
// pass, so the two 1-D passes equal the 2-D window sum.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fhd_internal.h"

namespace fhd {
namespace {

constexpr int RT = 256;       // threads per block
constexpr int MAXS_T = 32;    // radii with unrolled register-window kernels
constexpr int R_ROW = 8;      // outputs per thread, row pass
constexpr int R_COL = 8;      // outputs per thread, column pass
constexpr int TXC = 64;       // column-pass tile width
constexpr int TYC = R_COL * (RT / TXC);   // column-pass tile height
constexpr int CG = 4;         // channels per column-pass group
constexpr int RHO_INLINE = 8; // guides up to this dimension get inline weights

struct FA {
    const float* f;
    const float* p;
    const float* mu;    // K x rho
    const float* P;     // K x K, symmetric (least-squares coefficients)
    const float* Bpl;   // K planes of b, or null (weights computed inline)
    const float* Cpl;   // K planes of c, or null
    const int* labels;  // hard assignment
    float* planes;      // K(n+1) row-filtered planes, pitch Wp, S zero rows above and below
    float* out;
    float* den;
    // adjoint
    int fmode;          // row pass vector: 0 = [f, 1], 1 = [G / r, -(G . g_hat) / r]
    int factor_b;       // row pass factor: 0 = c (or b for the hard variant), 1 = b
    const float* gout;  // G = dL/dg_hat (n planes)
    const float* gimg;  // g_hat (n planes)
    const float* gden;  // r_hat
    float* beta;        // K planes
    float* gamma;       // K planes
    float* gradf;       // n planes or null
    const float* Md;    // dA^+/dsigma_r (K x K), batched adjoint
    float* gradp;       // rho planes or null, batched adjoint
    int n, rho, K, H, W, Wp, S, coef, tx, xcd_groups;
    int gsplit;         // column pass: blocks sharing one tile's channel groups
    long long N, Np;    // pixels; stride of the B / C planes
    long long Pp;       // stride of the intermediate planes: H + 2S rows of Wp, row y at y + S
    float inv2s2;       // 1 / (2 sigma_r^2), 0 for sigma_r = inf
    float* betas;       // adjoint, dL/dsigma_s: K planes of Y . (d omega / d sigma_s) * (c_l [f, 1]), or null
    float* Csave;       // row pass with inline weights: also store c_l of the block's own pixels (K planes), or null
    int bacc;           // adjoint column pass: add to the output planes instead of overwriting
    float w[FHD_MAX_RADIUS + 1];   // 1-D spatial taps w[|j|]
    float wd[FHD_MAX_RADIUS + 1];  // their derivative d w[|j|] / d sigma_s = w j^2 / sigma_s^3
    float yc[4];        // recursive Gaussian: B, b1/b0, b2/b0, b3/b0
};

// LDS skew: one pad word after every R_ROW = 8 entries.  A thread's window
// starting at h0 = 8 seg sits at 9 seg + q + q / 8, so a run of lanes reads
// with stride 9 words (no bank conflicts) at compile-time offsets from one base.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }

// ---------------------------------------------------------------------------
// Row pass, phase 1: the convolved factor g_l (c_l or b_l) and f on the halo
// run [x0 - S, x0 + tx + S) of row y, zero outside the image, into LDS:
//   cs[l * csp + pidx(h)], fs[ch * csp + pidx(h)].
// Inline weights (rho <= RHO_INLINE, K <= KMAX_INLINE): b_m = phi(mu_m - p)
// for every halo pixel and center, and c = A^+ b on the matrix cores.
constexpr int KMAX_INLINE = 32;

typedef float f32x16 __attribute__((ext_vector_type(16)));

// c = A^+ b for 32 consecutive pixels of a run on the matrix cores, one wave:
// C[i][l] = sum_m b_m(pixel i) A^+[m][l] as ceil(K / 2) steps of a 32 x 32 x 2
// FP32 product.  Lane j supplies b for pixel j % 32 and center 2s + j / 32
// (the A operand of step s) and A^+[2s + j / 32][j % 32] (the B operand, from
// the copy sP, zero outside the K x K block); it receives C[i][j % 32] for
// the 16 rows i = 8 (r / 4) + 4 (j / 32) + r % 4, r < 16.  The step body has
// no lane-dependent branch (centers past K read zero rows and are masked by
// a select), so the accumulator stays in the matrix registers across steps.
// RH: guide dimensions summed (entries past rho are zero on both sides).
template <int RH>
__device__ __forceinline__ f32x16 inline_coef_mfma(const FA& a, const float (&pr)[RH], bool in,
                                                   const float* smu, const float* sP) {
    const int kh = (threadIdx.x & 63) >> 5, pl = threadIdx.x & 31;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const int steps = (a.K + 1) >> 1;  // uniform
    for (int s = 0; s < steps; ++s) {
        const int m = 2 * s + kh;
        float d2 = 0.0f;
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            const float d = pr[r] - smu[m * RHO_INLINE + r];
            d2 = fmaf(d, d, d2);
        }
        const float e = __expf(-d2 * a.inv2s2);
        const float b = (in && m < a.K) ? e : 0.0f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b, sP[m * KMAX_INLINE + pl], acc, 0, 0, 0);
    }
    return acc;
}

// c = A^+ b for the run of 32 halo pixels from g0 (one wave), into cs; pr
// holds the guide at pixel g0 + (lane % 32).
template <int RH>
__device__ __forceinline__ void coef_run(const FA& a, int g0, bool in, const float (&pr)[RH], int hw, int csp,
                                         float* cs, const float* smu, const float* sP) {
    const int lane = threadIdx.x & 63, pl = lane & 31, kh = lane >> 5;
    // guides of at most 4 dimensions sum 4 entries per distance (the first 4
    // of pr; the rest are zero)
    const f32x16 acc = a.rho <= 4 ? inline_coef_mfma<4>(a, reinterpret_cast<const float(&)[4]>(pr), in, smu, sP)
                                  : inline_coef_mfma<RH>(a, pr, in, smu, sP);
    if (pl < a.K) {
        if (g0 + 32 <= hw) {  // uniform: a full run of 32 pixels
#pragma unroll
            for (int r = 0; r < 16; ++r) cs[pl * csp + pidx(g0 + 8 * (r >> 2) + 4 * kh + (r & 3))] = acc[r];
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int hh = g0 + 8 * (r >> 2) + 4 * kh + (r & 3);
                if (hh < hw) cs[pl * csp + pidx(hh)] = acc[r];
            }
        }
    }
}

// b_m of one halo pixel for every center, into cs (the hard variant's
// factor, and the adjoint's b_l Y).
template <int RH>
__device__ __forceinline__ void bfactor_loop(const FA& a, int h, bool in, const float (&pr)[RH], int csp, float* cs,
                                             const float* smu) {
    for (int m = 0; m < a.K; ++m) {
        float d2 = 0.0f;
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            const float d = pr[r] - smu[m * RHO_INLINE + r];
            d2 = fmaf(d, d, d2);
        }
        cs[m * csp + pidx(h)] = in ? __expf(-d2 * a.inv2s2) : 0.0f;
    }
}

template <int RH>
__device__ __forceinline__ void bfactor_pixel(const FA& a, int h, bool in, const float (&pr)[RH], int csp, float* cs,
                                              const float* smu) {
    if (a.rho <= 4)
        bfactor_loop<4>(a, h, in, reinterpret_cast<const float(&)[4]>(pr), csp, cs, smu);
    else
        bfactor_loop<RH>(a, h, in, pr, csp, cs, smu);
}

template <int RH>
__device__ __forceinline__ void guide_load(const FA& a, long long rowoff, int x, bool in, float (&pr)[RH]) {
#pragma unroll
    for (int r = 0; r < RH; ++r) pr[r] = (in && r < a.rho) ? a.p[(long long)r * a.N + rowoff + x] : 0.0f;
}

// The vector entries of one halo pixel: [f, 1] (fmode 0) or the adjoint
// vector [G / r, -(G . g_hat) / r] (fmode 1).  The loads of the first PF
// channels (v: f or G, u: g_hat, dn: r) are issued with the phase's other
// loads; the store forms the entries, loading channels past PF itself.
constexpr int PF = 4;

__device__ __forceinline__ void vec_load(const FA& a, long long rowoff, int x, bool in, float (&v)[PF],
                                         float (&u)[PF], float& dn) {
    const float* src = a.fmode == 0 ? a.f : a.gout;
#pragma unroll
    for (int ch = 0; ch < PF; ++ch) v[ch] = (in && ch < a.n) ? src[(long long)ch * a.N + rowoff + x] : 0.0f;
#pragma unroll
    for (int ch = 0; ch < PF; ++ch)
        u[ch] = (in && ch < a.n && a.fmode != 0) ? a.gimg[(long long)ch * a.N + rowoff + x] : 0.0f;
    dn = (in && a.fmode != 0) ? a.gden[rowoff + x] : 1.0f;
}

__device__ __forceinline__ void vec_store(const FA& a, long long rowoff, int h, int x, bool in, int csp, float* fs,
                                          const float (&v)[PF], const float (&u)[PF], float dn) {
    const int n = a.n;
    if (a.fmode == 0) {
#pragma unroll
        for (int ch = 0; ch < PF; ++ch)
            if (ch < n) fs[ch * csp + pidx(h)] = v[ch];
        for (int ch = PF; ch < n; ++ch) fs[ch * csp + pidx(h)] = in ? a.f[(long long)ch * a.N + rowoff + x] : 0.0f;
        fs[n * csp + pidx(h)] = in ? 1.0f : 0.0f;
    } else {
        const float inv = in ? 1.0f / dn : 0.0f;
        float dr = 0.0f;
#pragma unroll
        for (int ch = 0; ch < PF; ++ch)
            if (ch < n) {
                fs[ch * csp + pidx(h)] = v[ch] * inv;
                dr = fmaf(v[ch], u[ch], dr);
            }
        for (int ch = PF; ch < n; ++ch) {
            const float gv = in ? a.gout[(long long)ch * a.N + rowoff + x] : 0.0f;
            fs[ch * csp + pidx(h)] = gv * inv;
            dr = fmaf(gv, in ? a.gimg[(long long)ch * a.N + rowoff + x] : 0.0f, dr);
        }
        fs[n * csp + pidx(h)] = -dr * inv;
    }
}

// Row pass, phase 1: the convolved factor g_l (c_l or b_l) and the vector
// entries on the halo run [x0 - S, x0 + hw - S) of row y, zero outside the
// image, into LDS: cs[l * csp + pidx(h)], fs[ch * csp + pidx(h)].  Every
// global load of the phase is issued before the first LDS store (one round
// trip to memory instead of one per loop): the thread's halo pixel h = t,
// the zero-padded constants (KMAX_INLINE x RHO_INLINE centers, KMAX_INLINE x
// KMAX_INLINE A^+), and the guide at the pixels whose factors the thread
// forms (pixel t for b; the pixels of its wave's two 32-pixel runs for c).
// Halo runs longer than the block take the remaining pixels in loops.
template <int RH>
__device__ __forceinline__ void row_factors_rh(const FA& a, int y, int x0, int hw, int csp, float* cs, float* fs,
                                               float* smu, float* sP) {
    static_assert(KMAX_INLINE * RHO_INLINE == RT && KMAX_INLINE * KMAX_INLINE == 4 * RT,
                  "the constants' copies take one and four entries per thread");
    const int K = a.K, rho = a.rho;
    const long long rowoff = (long long)y * a.W;
    const int t = threadIdx.x, wave = t >> 6, pl = t & 31;
    const bool inl = a.Bpl == nullptr;
    const bool bfac = a.coef == FHD_COEF_HARD || a.factor_b;  // the factor is b itself
    const int x = x0 - a.S + t;
    const bool in = t < hw && x >= 0 && x < a.W;
    float v[PF], u[PF], dn;
    vec_load(a, rowoff, x, in, v, u, dn);
    float muv = 0.0f, pv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float pr[2][RH];
    bool gin[2] = {false, false};
    if (inl) {
        {
            const int m = t / RHO_INLINE, r = t - m * RHO_INLINE;
            muv = (m < K && r < rho) ? a.mu[m * rho + r] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + q * RT, m = e / KMAX_INLINE, l = e - m * KMAX_INLINE;
            pv[q] = (m < K && l < K) ? a.P[m * K + l] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int gh = bfac ? (k == 0 ? t : hw) : wave * 32 + k * 128 + pl;
            const int xx = x0 - a.S + gh;
            gin[k] = gh < hw && xx >= 0 && xx < a.W;
            guide_load<RH>(a, rowoff, xx, gin[k], pr[k]);
        }
    }
    if (t < hw) vec_store(a, rowoff, t, x, in, csp, fs, v, u, dn);
    for (int h = t + RT; h < hw; h += RT) {
        const int xh = x0 - a.S + h;
        const bool ih = xh >= 0 && xh < a.W;
        float v2[PF], u2[PF], d2;
        vec_load(a, rowoff, xh, ih, v2, u2, d2);
        vec_store(a, rowoff, h, xh, ih, csp, fs, v2, u2, d2);
    }
    if (!inl) {  // weights materialised by the weights pass
        const float* src = bfac ? a.Bpl : a.Cpl;
        const long long prow = (long long)y * a.Wp;
        for (int e = t; e < hw * K; e += RT) {
            const int l = e / hw, h = e - l * hw;
            const int xh = x0 - a.S + h;
            const bool ih = xh >= 0 && xh < a.W;
            cs[l * csp + pidx(h)] = ih ? src[(long long)l * a.Np + prow + xh] : 0.0f;
        }
        __syncthreads();
        return;
    }
    smu[t] = muv;
#pragma unroll
    for (int q = 0; q < 4; ++q) sP[t + q * RT] = pv[q];
    __syncthreads();
    if (bfac) {
        if (t < hw) bfactor_pixel<RH>(a, t, gin[0], pr[0], csp, cs, smu);
        for (int h = t + RT; h < hw; h += RT) {
            const int xh = x0 - a.S + h;
            const bool ih = xh >= 0 && xh < a.W;
            float p2[RH];
            guide_load<RH>(a, rowoff, xh, ih, p2);
            bfactor_pixel<RH>(a, h, ih, p2, csp, cs, smu);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int g0 = wave * 32 + k * 128;
            if (g0 < hw) coef_run<RH>(a, g0, gin[k], pr[k], hw, csp, cs, smu, sP);  // uniform per wave
        }
        for (int g0 = wave * 32 + 256; g0 < hw; g0 += 128) {
            const int xh = x0 - a.S + g0 + pl;
            const bool ih = g0 + pl < hw && xh >= 0 && xh < a.W;
            float p2[RH];
            guide_load<RH>(a, rowoff, xh, ih, p2);
            coef_run<RH>(a, g0, ih, p2, hw, csp, cs, smu, sP);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void row_factors(const FA& a, int y, int x0, int hw, int csp, float* cs, float* fs, float* smu,
                            float* sP) {
    row_factors_rh<RHO_INLINE>(a, y, x0, hw, csp, cs, fs, smu, sP);
}

__device__ __forceinline__ void store_row(const FA& a, float* dst, int x, const float* o, int R) {
    // dst points at (plane, row y, column 0)
    if (x + R <= a.W && (a.Wp & 3) == 0 && (R & 3) == 0) {
        for (int t = 0; t < R; t += 4)
            *reinterpret_cast<float4*>(dst + x + t) = make_float4(o[t], o[t + 1], o[t + 2], o[t + 3]);
    } else {
        for (int t = 0; t < R; ++t)
            if (x + t < a.W) dst[x + t] = o[t];
    }
}

// The S zero rows above and below every intermediate plane are written by
// the row pass itself: its grid has H + 2S rows, and a block of an outside
// row stores zeros over its column run in all K(n+1) planes.
__device__ __forceinline__ bool row_halo(const FA& a, int S, int by, int& y, int x0) {
    y = by - S;
    if (y >= 0 && y < a.H) return false;
    const int w = min(a.tx, a.W - x0);
    const int planes = a.K * (a.n + 1);
    float* row = a.planes + (long long)(y + S) * a.Wp + x0;
    for (int t = threadIdx.x; t < planes * w; t += RT) {
        const int pl = t / w, x = t - pl * w;
        row[(long long)pl * a.Pp + x] = 0.0f;
    }
    return true;
}

// The coefficients c_l of the block's own pixels (halo index S + h), kept
// for the adjoint when the call saves its intermediates.
__device__ __forceinline__ void row_save_coefs(const FA& a, int y, int x0, int S, int csp, const float* cs) {
    if (a.Csave == nullptr) return;
    const int w = min(a.tx, a.W - x0);
    float* dst = a.Csave + (long long)y * a.Wp + x0;
    for (int t = threadIdx.x; t < a.K * w; t += RT) {
        const int l = t / w, h = t - l * w;
        dst[(long long)l * a.Np + h] = cs[l * csp + pidx(S + h)];
    }
}

// Gaussian row pass, radius S known at compile time: each task filters R
// outputs of one cluster from a register window of R + 2S inputs.
template <int S>
__device__ __forceinline__ void row_gauss_body(const FA& a, int bx, int by) {
    extern __shared__ float lds[];
    constexpr int R = R_ROW;
    constexpr int WIN = R + 2 * S;
    const int x0 = bx * a.tx;
    int y;
    if (row_halo(a, S, by, y, x0)) return;
    const int hw = a.tx + 2 * S;
    const int csp = pidx(hw - 1) + 1;
    float* cs = lds;
    float* fs = cs + a.K * csp;
    float* smu = fs + (a.n + 1) * csp;
    float* sP = smu + KMAX_INLINE * RHO_INLINE;
    row_factors(a, y, x0, hw, csp, cs, fs, smu, sP);
    row_save_coefs(a, y, x0, S, csp, cs);
    const int nseg = a.tx / R;
    const int n = a.n;
    for (int task = threadIdx.x; task < a.K * nseg; task += RT) {
        const int l = task / nseg, seg = task - l * nseg;
        const int x = x0 + seg * R;
        if (x >= a.W) continue;
        float cw[WIN];
        static_assert(R == 8, "the LDS skew assumes 8 outputs per task");
        const int wb = seg * (R + 1);  // pidx(seg * R)
#pragma unroll
        for (int q = 0; q < WIN; ++q) cw[q] = cs[l * csp + wb + q + (q >> 3)];
        float o[R];
        if (a.fmode == 0) {  // last vector entry: the constant 1
#pragma unroll
            for (int t = 0; t < R; ++t) {
                float s = a.w[0] * cw[t + S];
#pragma unroll
                for (int j = 1; j <= S; ++j) s = fmaf(a.w[j], cw[t + S - j] + cw[t + S + j], s);
                o[t] = s;
            }
        } else {
            float u[WIN];
#pragma unroll
            for (int q = 0; q < WIN; ++q) u[q] = cw[q] * fs[n * csp + wb + q + (q >> 3)];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                float s = a.w[0] * u[t + S];
#pragma unroll
                for (int j = 1; j <= S; ++j) s = fmaf(a.w[j], u[t + S - j] + u[t + S + j], s);
                o[t] = s;
            }
        }
        const long long rowp = (long long)(y + S) * a.Wp;
        float* base = a.planes + (long long)l * (n + 1) * a.Pp + rowp;
        store_row(a, base + (long long)n * a.Pp, x, o, R);
        for (int ch = 0; ch < n; ++ch) {
            float u[WIN];
#pragma unroll
            for (int q = 0; q < WIN; ++q) u[q] = cw[q] * fs[ch * csp + wb + q + (q >> 3)];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                float s = a.w[0] * u[t + S];
#pragma unroll
                for (int j = 1; j <= S; ++j) s = fmaf(a.w[j], u[t + S - j] + u[t + S + j], s);
                o[t] = s;
            }
            store_row(a, base + (long long)ch * a.Pp, x, o, R);
        }
    }
}

// Batched launches: the blocks of image b of a ragged batch are
// [pre[b], pre[b + 1]) of one 1-D grid; the image's parameters are fas[b].
__device__ __forceinline__ int batch_block(const int* __restrict__ pre, int B, int& b) {
    const int blk = (int)blockIdx.x;
    int i = 0;
    while (i + 1 < B && blk >= pre[i + 1]) ++i;  // uniform per block, B small
    b = i;
    return blk - pre[i];
}

template <int S>
__global__ __launch_bounds__(RT) void row_gauss(FA a) {
    row_gauss_body<S>(a, (int)blockIdx.x, (int)blockIdx.y);
}

template <int S>
__global__ __launch_bounds__(RT) void row_gauss_batch(const FA* __restrict__ fas, const int* __restrict__ pre,
                                                      int B) {
    int b;
    const int t = batch_block(pre, B, b);
    const FA& a = fas[b];
    const int gx = (a.W + a.tx - 1) / a.tx;
    row_gauss_body<S>(a, t % gx, t / gx);
}

// Row pass for any radius: box kernel as a running sum, Gaussian tap by tap.
template <bool BOX>
__global__ __launch_bounds__(RT) void row_generic(FA a) {
    extern __shared__ float lds[];
    constexpr int R = 16;
    const int S = a.S;
    const int x0 = blockIdx.x * a.tx;
    int y;
    if (row_halo(a, S, (int)blockIdx.y, y, x0)) return;
    const int hw = a.tx + 2 * S;
    const int csp = pidx(hw - 1) + 1;
    float* cs = lds;
    float* fs = cs + a.K * csp;
    float* smu = fs + (a.n + 1) * csp;
    float* sP = smu + KMAX_INLINE * RHO_INLINE;
    row_factors(a, y, x0, hw, csp, cs, fs, smu, sP);
    const int nseg = a.tx / R;
    const int n = a.n;
    for (int task = threadIdx.x; task < a.K * nseg * (n + 1); task += RT) {
        const int ch = task % (n + 1);
        const int rest = task / (n + 1);
        const int l = rest / nseg, seg = rest - l * nseg;
        const int x = x0 + seg * R;
        if (x >= a.W) continue;
        const float* cl = cs + l * csp;
        const float* fc = fs + ch * csp;
        auto U = [&](int h) { return (ch < n || a.fmode != 0) ? cl[pidx(h)] * fc[pidx(h)] : cl[pidx(h)]; };
        float o[R];
        const int h0 = seg * R;  // halo index of the window start for output x
        if (BOX) {  // running sum in FP64, as in row_box
            double s = 0.0;
            for (int q = 0; q <= 2 * S; ++q) s += (double)U(h0 + q);
            o[0] = (float)s;
#pragma unroll
            for (int t = 1; t < R; ++t) {
                s += (double)U(h0 + t + 2 * S) - (double)U(h0 + t - 1);
                o[t] = (float)s;
            }
        } else {
#pragma unroll
            for (int t = 0; t < R; ++t) {
                float s = a.w[0] * U(h0 + t + S);
                for (int j = 1; j <= S; ++j) s = fmaf(a.w[j], U(h0 + t + S - j) + U(h0 + t + S + j), s);
                o[t] = s;
            }
        }
        float* dst = a.planes + ((long long)l * (n + 1) + ch) * a.Pp + (long long)(y + S) * a.Wp;
        store_row(a, dst, x, o, R);
    }
}

// ---------------------------------------------------------------------------
// Box row pass, any radius: the window sums of u = g_l [f, 1] along the halo
// run as running sums, the O(1) box convolution of Sec. II-C.  A wave takes
// CH_BOX vector entries of one cluster l (one read of g_l serves them all,
// and their scans are independent); lane i takes the RB_BOX consecutive
// outputs o = c0 + RB_BOX i + t of a chunk of 64 RB_BOX.  With the
// differences d(o) = u(o + 2S) - u(o - 1), the window sum at o is the sum at
// the chunk's first output plus the inclusive prefix of d over the chunk: a
// scan within the lane, then one across the wave with DPP row shifts and row
// broadcasts.  The first window sum is a wave reduction of u(0 .. 2S); each
// chunk hands its last sum to the next.  The work per output does not grow
// with S.  The sums run in FP64 (the vector units issue FP64 adds at the
// FP32 rate; the differences of FP32 products are exact in FP64) and each
// output is rounded to FP32 once, so a window sum carries the rounding of its
// own terms only, not that of the larger sums the scan passed on its way.
constexpr int RB_BOX = 4;
constexpr int CH_BOX = 4;

// v of the lane that the DPP control CTRL names; 0 where that lane lies
// outside the row (or the wave) or the lane's row is not in the mask ROWS
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_in(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// inclusive prefix sums over the 64 lanes of the wave (all lanes active), of
// CH_BOX independent values per lane
__device__ __forceinline__ void wave_scan(double (&v)[CH_BOX]) {
#pragma unroll
    for (int c = 0; c < CH_BOX; ++c) v[c] += dpp_in<0x111, 0xF>(v[c]);  // row_shr:1
#pragma unroll
    for (int c = 0; c < CH_BOX; ++c) v[c] += dpp_in<0x112, 0xF>(v[c]);  // row_shr:2
#pragma unroll
    for (int c = 0; c < CH_BOX; ++c) v[c] += dpp_in<0x114, 0xF>(v[c]);  // row_shr:4
#pragma unroll
    for (int c = 0; c < CH_BOX; ++c) v[c] += dpp_in<0x118, 0xF>(v[c]);  // row_shr:8: prefix within rows of 16
#pragma unroll
    for (int c = 0; c < CH_BOX; ++c) v[c] += dpp_in<0x142, 0xA>(v[c]);  // row_bcast:15: rows 1, 3 add rows 0, 2
#pragma unroll
    for (int c = 0; c < CH_BOX; ++c) v[c] += dpp_in<0x143, 0xC>(v[c]);  // row_bcast:31: rows 2, 3 add lane 31
}

__device__ __forceinline__ double lane63(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ void row_box_body(const FA& a, int bx, int by) {
    extern __shared__ float lds[];
    const int S = a.S;
    const int x0 = bx * a.tx;
    int y;
    if (row_halo(a, S, by, y, x0)) return;
    const int hw = a.tx + 2 * S;
    const int csp = pidx(hw - 1) + 1;
    float* cs = lds;
    float* fs = cs + a.K * csp;
    float* smu = fs + (a.n + 1) * csp;
    float* sP = smu + KMAX_INLINE * RHO_INLINE;
    row_factors(a, y, x0, hw, csp, cs, fs, smu, sP);
    row_save_coefs(a, y, x0, S, csp, cs);
    const int n = a.n, w = min(a.tx, a.W - x0);
    const int lane = threadIdx.x & 63;
    const int chunks = (n + 1 + CH_BOX - 1) / CH_BOX;
    const long long rowp = (long long)(y + S) * a.Wp + x0;
    for (int task = threadIdx.x >> 6; task < a.K * chunks; task += RT / 64) {  // uniform per wave
        const int l = task / chunks, e0 = (task - l * chunks) * CH_BOX;
        const float* cl = cs + l * csp;
        // u of entry e0 + c at halo index h: g_l f_c, or g_l for the constant
        // last entry 1 of the forward vector (entries past n read as 0)
        auto U = [&](double (&u)[CH_BOX], int h) {
            const int ph = pidx(h);
            const float g = cl[ph];
#pragma unroll
            for (int c = 0; c < CH_BOX; ++c) {
                const int e = e0 + c;
                const float v = e > n ? 0.0f : (e < n || a.fmode != 0) ? g * fs[e * csp + ph] : g;
                u[c] = (double)v;
            }
        };
        double carry[CH_BOX];
#pragma unroll
        for (int c = 0; c < CH_BOX; ++c) carry[c] = 0.0;
        for (int q = lane; q <= 2 * S; q += 64) {
            double u[CH_BOX];
            U(u, q);
#pragma unroll
            for (int c = 0; c < CH_BOX; ++c) carry[c] += u[c];
        }
        wave_scan(carry);
#pragma unroll
        for (int c = 0; c < CH_BOX; ++c) carry[c] = lane63(carry[c]);  // the window sums at output 0
        float* dst = a.planes + ((long long)l * (n + 1) + e0) * a.Pp + rowp;
        for (int c0 = 0; c0 < w; c0 += 64 * RB_BOX) {
            const int ob = c0 + lane * RB_BOX;
            double d[RB_BOX][CH_BOX];
#pragma unroll
            for (int t = 0; t < RB_BOX; ++t) {
                const int o = ob + t;
                if (o >= 1 && o < w) {
                    double ui[CH_BOX], uo[CH_BOX];
                    U(ui, o + 2 * S);
                    U(uo, o - 1);
#pragma unroll
                    for (int c = 0; c < CH_BOX; ++c) d[t][c] = ui[c] - uo[c];
                } else {
#pragma unroll
                    for (int c = 0; c < CH_BOX; ++c) d[t][c] = 0.0;
                }
                if (t > 0) {
#pragma unroll
                    for (int c = 0; c < CH_BOX; ++c) d[t][c] += d[t - 1][c];
                }
            }
            double incl[CH_BOX];
#pragma unroll
            for (int c = 0; c < CH_BOX; ++c) incl[c] = d[RB_BOX - 1][c];
            wave_scan(incl);
            static_assert(RB_BOX == 4, "one float4 store per lane and entry");
#pragma unroll
            for (int c = 0; c < CH_BOX; ++c) {
                const double base = carry[c] + dpp_in<0x138, 0xF>(incl[c]);  // wave_shr:1: the lanes below
                float o4[RB_BOX];
#pragma unroll
                for (int t = 0; t < RB_BOX; ++t) o4[t] = (float)(base + d[t][c]);
                if (e0 + c <= n) {
                    float* dp = dst + (long long)c * a.Pp;
                    if (ob + RB_BOX <= w && (a.Wp & 3) == 0) {
                        *reinterpret_cast<float4*>(dp + ob) = make_float4(o4[0], o4[1], o4[2], o4[3]);
                    } else {
#pragma unroll
                        for (int t = 0; t < RB_BOX; ++t)
                            if (ob + t < w) dp[ob + t] = o4[t];
                    }
                }
                carry[c] += lane63(incl[c]);
            }
        }
    }
}

__global__ __launch_bounds__(RT) void row_box(FA a) { row_box_body(a, (int)blockIdx.x, (int)blockIdx.y); }

__global__ __launch_bounds__(RT) void row_box_batch(const FA* __restrict__ fas, const int* __restrict__ pre, int B) {
    int b;
    const int t = batch_block(pre, B, b);
    const FA& a = fas[b];
    const int gx = (a.W + a.tx - 1) / a.tx;
    row_box_body(a, t % gx, t / gx);
}

// ---------------------------------------------------------------------------
// Column pass with the recombination of eqs. (15)-(16) fused in.

struct ColTile {
    int x, y0, bx0, by0;
    bool block_active;  // the block maps to a tile
    bool active;        // this thread's column is inside the image
};

__device__ __forceinline__ ColTile col_tile(const FA& a, int ty, int blk) {
    // XCD-aware order: consecutive blocks on one XCD take vertically adjacent
    // tiles, so the S-row halos they share stay in that XCD's L2.  With a
    // split of the channel groups the grid repeats this order gsplit times.
    const int gx = (a.W + TXC - 1) / TXC, gy = (a.H + ty - 1) / ty;
    const int total = gx * gy;
    const int per = a.xcd_groups;  // blocks per XCD
    const int b = blk % (per * 8);
    const int t = (b & 7) * per + (b >> 3);
    ColTile c;
    c.block_active = t < total;
    const int bx = t / gy, by = t - bx * gy;
    c.bx0 = bx * TXC;
    c.by0 = by * ty;
    c.x = c.bx0 + (threadIdx.x & (TXC - 1));
    c.y0 = c.by0 + (threadIdx.x / TXC) * (ty / (RT / TXC));
    c.active = c.block_active && c.x < a.W;
    return c;
}

// Guide values of the tile's pixels (inline weights only): sp[r][row][col].
__device__ __forceinline__ void col_stage_guide(const FA& a, int bx0, int by0, int ty, float* sp) {
    if (a.Bpl != nullptr || a.coef == FHD_COEF_HARD) return;
    const int cnt = a.rho * ty * TXC;
    for (int t = threadIdx.x; t < cnt; t += RT) {
        const int r = t / (ty * TXC), rem = t - r * ty * TXC;
        const int yy = by0 + rem / TXC, xx = bx0 + (rem & (TXC - 1));
        sp[t] = (yy < a.H && xx < a.W) ? a.p[(long long)r * a.N + (long long)yy * a.W + xx] : 0.0f;
    }
}

// Recombination weight h_l of the R outputs of a thread: b_l(i) for the
// least-squares coefficients, the cluster indicator for the hard variant.
// Weight modes of the column pass.
enum { WM_INLINE = 0, WM_PLANES = 1, WM_HARD = 2 };

template <int R, int MODE>
__device__ __forceinline__ void recomb_weights(const FA& a, int l, int x, int y0, int ly0, int lx, int ty,
                                               const float* sp, const int (&lab)[R], float (&hl)[R]) {
    if (MODE == WM_HARD) {
#pragma unroll
        for (int t = 0; t < R; ++t) hl[t] = lab[t] == l ? 1.0f : 0.0f;
    } else if (MODE == WM_PLANES) {
        const float* bp = a.Bpl + (long long)l * a.Np + (long long)y0 * a.Wp + x;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            hl[t] = (y0 + t < a.H && x < a.W) ? *bp : 0.0f;
            bp += a.Wp;
        }
    } else {
        float d2[R];
#pragma unroll
        for (int t = 0; t < R; ++t) d2[t] = 0.0f;
        for (int r = 0; r < a.rho; ++r) {
            const float m = a.mu[l * a.rho + r];
            const float* row = sp + (r * ty + ly0) * TXC + lx;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const float d = row[t * TXC] - m;
                d2[t] = fmaf(d, d, d2[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) hl[t] = __expf(-d2[t] * a.inv2s2);
    }
}

template <int R, int MODE>
__device__ __forceinline__ void col_load_labels(const FA& a, int x, int y0, int (&lab)[R]) {
#pragma unroll
    for (int t = 0; t < R; ++t)
        lab[t] = (MODE == WM_HARD && y0 + t < a.H && x < a.W) ? a.labels[(long long)(y0 + t) * a.W + x] : -1;
}

template <int R>
__device__ __forceinline__ void col_finish(const FA& a, int x, int y0, int g, const float (&acc)[CG][R],
                                           float (&dv)[R]) {
    const int n = a.n;
    if (g == 0) {
#pragma unroll
        for (int t = 0; t < R; ++t) dv[t] = 1.0f / acc[0][t];
        if (a.den != nullptr) {
            float* dp = a.den + (long long)y0 * a.W + x;
            for (int t = 0; t < R && y0 + t < a.H; ++t) {
                *dp = acc[0][t];
                dp += a.W;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CG; ++c) {
        const int gi = g * CG + c;
        if (gi > n) break;
        if (gi == 0) continue;
        float* op = a.out + (long long)(gi - 1) * a.N + (long long)y0 * a.W + x;
        for (int t = 0; t < R && y0 + t < a.H; ++t) {
            *op = acc[c][t] * dv[t];
            op += a.W;
        }
    }
}

// Column pass.  A block owns a tile of TXC columns x ty rows; for every
// plane (cluster l, channel) in turn it stages the tile's rows plus the 2S
// halo rows in LDS (the next plane's rows are in flight from global memory
// into registers while the current one is filtered), and every thread
// filters R consecutive rows of one column from a register window.
__device__ __forceinline__ int plane_index(int n, int g, int l, int c) {
    const int gi = g * CG + c;
    return l * (n + 1) + (gi == 0 ? n : gi - 1);
}

// successor of (g, l, c) in the visiting order; false at the end
__device__ __forceinline__ bool plane_next(int n, int K, int& g, int& l, int& c) {
    const int groups = (n + 1 + CG - 1) / CG;
    ++c;
    if (c < CG && g * CG + c <= n) return true;
    c = 0;
    if (++l < K) return true;
    l = 0;
    return ++g < groups;
}

// Order in which a block of the column pass visits its planes (g, l, c):
// part p of a tile split gsplit ways takes the channel groups p, p + gsplit,
// ...; a part other than 0 first visits the normaliser plane (group 0,
// channel 0) of every cluster, so it can divide its own channels.
struct PlaneSeq {
    int n, K, groups, gsplit, part;
    __device__ void start(int& ph, int& g, int& l, int& c) const {
        ph = part == 0 ? 1 : 0;
        g = 0;
        l = 0;
        c = 0;
    }
    // successor of (ph, g, l, c); false at the end
    __device__ bool next(int& ph, int& g, int& l, int& c) const {
        if (ph == 0) {
            if (++l < K) return true;
            ph = 1;
            g = part;
            l = 0;
            c = 0;
            return g < groups;
        }
        ++c;
        if (c < CG && g * CG + c <= n) return true;
        c = 0;
        if (++l < K) return true;
        l = 0;
        g += gsplit;
        return g < groups;
    }
};

// The 1-D window of the column pass, as a policy of col_body: R outputs per
// thread, tiles of TY rows, PER staged values per thread and plane (the tile
// plus its 2S halo rows), and filter(), which forms a thread's R window sums
// from its column of the staged tile (tile row q = image row y0 - S + q).
//
// ColFir: taps w[|j|] at radius S known at compile time (Gaussian, or the box
// as unit taps), from a register window of R + 2S inputs.
template <int S>
struct ColFir {
    static constexpr int R = R_COL;
    static constexpr int TY = TYC;
    static constexpr int PER = ((TY + 2 * S) * TXC + RT - 1) / RT;
    __device__ static int rows(const FA&) { return TY + 2 * S; }
    __device__ static void filter(const FA& a, const float* col, float (&s)[R]) {
        constexpr int WIN = R + 2 * S;
        float win[WIN];
#pragma unroll
        for (int q = 0; q < WIN; ++q) win[q] = col[q * TXC];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            float v = a.w[0] * win[t + S];
#pragma unroll
            for (int j = 1; j <= S; ++j) v = fmaf(a.w[j], win[t + S - j] + win[t + S + j], v);
            s[t] = v;
        }
    }
};

// ColBox: the box window of any radius S <= SB as a running sum down the
// column (Sec. II-C): the first window sum directly, then one add and one
// subtract per output, in FP64 (as in the box row pass: each output carries
// the rounding of its own window's terms only).
template <int SB>
struct ColBox {
    static constexpr int R = R_COL;
    static constexpr int TY = TYC;
    static constexpr int PER = ((TY + 2 * SB) * TXC + RT - 1) / RT;
    __device__ static int rows(const FA& a) { return TY + 2 * a.S; }
    __device__ static void filter(const FA& a, const float* col, float (&s)[R]) {
        const int S2 = 2 * a.S;
        double v = 0.0;
#pragma unroll 4
        for (int q = 0; q <= S2; ++q) v += (double)col[q * TXC];
        s[0] = (float)v;
#pragma unroll
        for (int t = 1; t < R; ++t) {
            v += (double)col[(t + S2) * TXC] - (double)col[(t - 1) * TXC];
            s[t] = (float)v;
        }
    }
};

template <class F, int MODE>
__device__ __forceinline__ void col_body(const FA& a, int blk) {
    constexpr int R = F::R;
    constexpr int TY = F::TY;
    constexpr int PER = F::PER;  // staged values per thread and plane
    const int ROWS = F::rows(a);
    __shared__ float tbuf[PER * RT];
    extern __shared__ float sp[];
    const ColTile tile = col_tile(a, TY, blk);
    if (!tile.block_active) return;
    if (MODE == WM_INLINE) col_stage_guide(a, tile.bx0, tile.by0, TY, sp);
    const int n = a.n, K = a.K;
    const int lx = threadIdx.x & (TXC - 1), tr = threadIdx.x / TXC;
    const int x = tile.x, y0 = tile.y0;
    const int ly0 = tr * R;
    const int groups = (n + 1 + CG - 1) / CG;
    const PlaneSeq seq{n, K, groups, a.gsplit, blk / (a.xcd_groups * 8)};
    if (seq.part >= groups) return;
    // staging: thread loads rows tr, tr+4, ... of the tile at column lx
    const long long tile_off = (long long)tile.by0 * a.Wp + tile.bx0 + tr * (long long)a.Wp + lx;
    const long long step = (long long)(RT / TXC) * a.Wp;
    auto fetch = [&](int plane, float (&pre)[PER]) {
        const float* src = a.planes + (long long)plane * a.Pp + tile_off;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            pre[k] = (tr + k * (RT / TXC) < ROWS) ? *src : 0.0f;
            src += step;
        }
    };
    auto stash = [&](float* dst, const float (&pre)[PER]) {
#pragma unroll
        for (int k = 0; k < PER; ++k) dst[k * RT + threadIdx.x] = pre[k];
    };
    int lab[R];
    col_load_labels<R, MODE>(a, x, y0, lab);
    float pre[PER];
    int ph, sg, sl, sc;  // the plane staged next
    seq.start(ph, sg, sl, sc);
    fetch(plane_index(n, sg, sl, sc), pre);
    stash(tbuf, pre);
    __syncthreads();
    // filter the staged plane (tile row ly0 + q holds image row y0 - S + q)
    // into s and queue the following one
    auto filter_plane = [&](float (&s)[R]) {
        int nph = ph, ng = sg, nl = sl, nc = sc;
        const bool more = seq.next(nph, ng, nl, nc);
        if (more) fetch(plane_index(n, ng, nl, nc), pre);
        F::filter(a, tbuf + ly0 * TXC + lx, s);
        // one LDS copy of a plane: the next plane waits in registers while
        // this one is filtered
        __syncthreads();
        if (more) stash(tbuf, pre);
        __syncthreads();
        ph = nph;
        sg = ng;
        sl = nl;
        sc = nc;
    };
    auto consume = [&](const float (&hl)[R], float (&acc)[R]) {
        float s[R];
        filter_plane(s);
#pragma unroll
        for (int t = 0; t < R; ++t) acc[t] = fmaf(hl[t], s[t], acc[t]);
    };
    float dv[R];
    if (seq.part != 0) {  // the normaliser, for this part's own division
        float ad[R];
#pragma unroll
        for (int t = 0; t < R; ++t) ad[t] = 0.0f;
        for (int l = 0; l < K; ++l) {
            float hl[R];
            recomb_weights<R, MODE>(a, l, x, y0, ly0, lx, TY, sp, lab, hl);
            consume(hl, ad);
        }
#pragma unroll
        for (int t = 0; t < R; ++t) dv[t] = 1.0f / ad[t];
    }
    for (int g = seq.part; g < groups; g += seq.gsplit) {
        float acc[CG][R];
#pragma unroll
        for (int c = 0; c < CG; ++c)
#pragma unroll
            for (int t = 0; t < R; ++t) acc[c][t] = 0.0f;
        const int nc = min(CG, n + 1 - g * CG);  // channels of this group
        for (int l = 0; l < K; ++l) {
            float hl[R];
            recomb_weights<R, MODE>(a, l, x, y0, ly0, lx, TY, sp, lab, hl);
            if constexpr (MODE != WM_PLANES) {
                // the channel loop unrolled, each channel's accumulator
                // fixed; the barriers inside filter_plane keep the next
                // window's LDS reads after this one's FIR, so one window is
                // live at a time
#pragma unroll
                for (int c = 0; c < CG; ++c) {
                    if (c < nc) {  // uniform
                        float s[R];
                        filter_plane(s);
#pragma unroll
                        for (int t = 0; t < R; ++t) acc[c][t] = fmaf(hl[t], s[t], acc[c][t]);
                    }
                }
            } else {
                // with weight planes the unrolled loop takes 145-161 VGPRs
                // (three waves per SIMD instead of four) and measured slower
                // on the 32-band image: one copy of the plane loop, a
                // uniform switch picking the accumulator
#pragma unroll 1
                for (int c = 0; c < nc; ++c) {
                    float s[R];
                    filter_plane(s);
                    switch (c) {
                        case 0:
#pragma unroll
                            for (int t = 0; t < R; ++t) acc[0][t] = fmaf(hl[t], s[t], acc[0][t]);
                            break;
                        case 1:
#pragma unroll
                            for (int t = 0; t < R; ++t) acc[1][t] = fmaf(hl[t], s[t], acc[1][t]);
                            break;
                        case 2:
#pragma unroll
                            for (int t = 0; t < R; ++t) acc[2][t] = fmaf(hl[t], s[t], acc[2][t]);
                            break;
                        default:
#pragma unroll
                            for (int t = 0; t < R; ++t) acc[3][t] = fmaf(hl[t], s[t], acc[3][t]);
                            break;
                    }
                }
            }
        }
        if (tile.active) col_finish<R>(a, x, y0, g, acc, dv);
    }
}

template <int S, int MODE>
__global__ __launch_bounds__(RT) void col_gauss(FA a) {
    col_body<ColFir<S>, MODE>(a, (int)blockIdx.x);
}

template <int S, int MODE>
__global__ __launch_bounds__(RT) void col_gauss_batch(const FA* __restrict__ fas, const int* __restrict__ pre,
                                                      int B) {
    int b;
    const int t = batch_block(pre, B, b);
    col_body<ColFir<S>, MODE>(fas[b], t);
}

template <int SB, int MODE>
__global__ __launch_bounds__(RT) void col_box(FA a) {
    col_body<ColBox<SB>, MODE>(a, (int)blockIdx.x);
}

template <int SB, int MODE>
__global__ __launch_bounds__(RT) void col_box_batch(const FA* __restrict__ fas, const int* __restrict__ pre, int B) {
    int b;
    const int t = batch_block(pre, B, b);
    col_body<ColBox<SB>, MODE>(fas[b], t);
}

// Column pass for any radius (box as a running sum, Gaussian tap by tap),
// single-buffered tile in dynamic LDS after the guide tile.
template <bool BOX, int MODE>
__global__ __launch_bounds__(RT) void col_generic(FA a) {
    constexpr int R = 16;
    constexpr int TY = R * (RT / TXC);
    extern __shared__ float sp[];
    const ColTile tile = col_tile(a, TY, (int)blockIdx.x);
    if (!tile.block_active) return;
    if (MODE == WM_INLINE) col_stage_guide(a, tile.bx0, tile.by0, TY, sp);
    __syncthreads();  // every wave reads guide rows staged by the others
    float* tb = sp + (MODE == WM_INLINE ? a.rho * TY * TXC : 0);
    const int n = a.n, K = a.K, S = a.S;
    const int rows = TY + 2 * S;
    const int lx = threadIdx.x & (TXC - 1), tr = threadIdx.x / TXC;
    const int x = tile.x, y0 = tile.y0;
    const int ly0 = tr * R;
    int lab[R];
    col_load_labels<R, MODE>(a, x, y0, lab);
    const int groups = (n + 1 + CG - 1) / CG;
    float dv[R];
    for (int g = 0; g < groups; ++g) {
        float acc[CG][R];
#pragma unroll
        for (int c = 0; c < CG; ++c)
#pragma unroll
            for (int t = 0; t < R; ++t) acc[c][t] = 0.0f;
        for (int l = 0; l < K; ++l) {
            float hl[R];
            recomb_weights<R, MODE>(a, l, x, y0, ly0, lx, TY, sp, lab, hl);
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                if (g * CG + c > n) break;
                const int plane = plane_index(n, g, l, c);
                __syncthreads();  // previous plane fully consumed
                const float* src = a.planes + (long long)plane * a.Pp + (long long)tile.by0 * a.Wp + tile.bx0;
                for (int e = threadIdx.x; e < rows * TXC; e += RT)
                    tb[e] = src[(long long)(e / TXC) * a.Wp + (e & (TXC - 1))];
                __syncthreads();
                const float* col = tb + ly0 * TXC + lx;  // tile row ly0 + q = image row y0 - S + q
                if (BOX) {  // running sum in FP64, as in ColBox
                    double s = 0.0;
                    for (int q = 0; q <= 2 * S; ++q) s += (double)col[q * TXC];
                    acc[c][0] = fmaf(hl[0], (float)s, acc[c][0]);
#pragma unroll
                    for (int t = 1; t < R; ++t) {
                        s += (double)col[(t + 2 * S) * TXC] - (double)col[(t - 1) * TXC];
                        acc[c][t] = fmaf(hl[t], (float)s, acc[c][t]);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        float s = a.w[0] * col[(t + S) * TXC];
                        for (int j = 1; j <= S; ++j)
                            s = fmaf(a.w[j], col[(t + S - j) * TXC] + col[(t + S + j) * TXC], s);
                        acc[c][t] = fmaf(hl[t], s, acc[c][t]);
                    }
                }
            }
        }
        if (tile.active) col_finish<R>(a, x, y0, g, acc, dv);
    }
}

// ---------------------------------------------------------------------------
// Adjoint column passes.  Same staging and filtering as the forward column
// pass; the epilogue per cluster l and pixel i is
//   BETA:  beta_l(i)  = Y(i) . Q_l(i),  Y = [G / r, -(G . g_hat) / r]
//          (Q_l = w * (c_l [f, 1]) recomputed: dL/db_l from the recombination)
//   GAMMA: gamma_l(i) = [f(i), 1] . Z_l(i)  and  dL/df(i) += c_l(i) Z_l(i)[0:n]
//          (Z_l = w * (b_l Y): the adjoint of the convolution applied to
//          dL/dQ_l = b_l Y; w is symmetric and zero-extended, so its adjoint is
//          itself)
// AM_BETAS: AM_BETA plus, for dL/dsigma_s, the same planes filtered with the
// derivative taps (the column factor of d omega / d sigma_s) into a.betas
enum { AM_BETA = 0, AM_GAMMA = 1, AM_BETAS = 2 };

template <int S, int MODE>
__device__ __forceinline__ void col_adj_body(const FA& a, int blk) {
    constexpr int R = R_COL;
    constexpr int TY = TYC;
    constexpr int ROWS = TY + 2 * S;
    constexpr int PER = (ROWS * TXC + RT - 1) / RT;
    constexpr int WIN = R + 2 * S;
    __shared__ float tbuf[PER * RT];
    const ColTile tile = col_tile(a, TY, blk);
    if (!tile.block_active) return;
    const int n = a.n, K = a.K;
    const int lx = threadIdx.x & (TXC - 1), tr = threadIdx.x / TXC;
    const int x = tile.x, y0 = tile.y0;
    const int ly0 = tr * R;
    const long long tile_off = (long long)tile.by0 * a.Wp + tile.bx0 + tr * (long long)a.Wp + lx;
    const long long step = (long long)(RT / TXC) * a.Wp;
    auto fetch = [&](int plane, float (&pre)[PER]) {
        const float* src = a.planes + (long long)plane * a.Pp + tile_off;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            pre[k] = (tr + k * (RT / TXC) < ROWS) ? *src : 0.0f;
            src += step;
        }
    };
    auto stash = [&](float* dst, const float (&pre)[PER]) {
#pragma unroll
        for (int k = 0; k < PER; ++k) dst[k * RT + threadIdx.x] = pre[k];
    };
    float pre[PER];
    fetch(plane_index(n, 0, 0, 0), pre);
    stash(tbuf, pre);
    __syncthreads();
    const int groups = (n + 1 + CG - 1) / CG;
    const bool act = tile.active;
    for (int g = 0; g < groups; ++g) {
        // the group's entries of the per-pixel vector (Y for BETA, [f, 1] for GAMMA)
        float vec[CG][R];
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            const int gi = g * CG + c;
            const int ch = gi == 0 ? n : gi - 1;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                float v = 0.0f;
                if (act && gi <= n && y0 + t < a.H) {
                    const long long off = (long long)(y0 + t) * a.W + x;
                    if (MODE != AM_GAMMA) {
                        const float inv = 1.0f / a.gden[off];
                        if (ch < n) {
                            v = a.gout[(long long)ch * a.N + off] * inv;
                        } else {
                            float dr = 0.0f;
                            for (int q = 0; q < n; ++q)
                                dr = fmaf(a.gout[(long long)q * a.N + off], a.gimg[(long long)q * a.N + off], dr);
                            v = -dr * inv;
                        }
                    } else {
                        v = ch < n ? a.f[(long long)ch * a.N + off] : 1.0f;
                    }
                }
                vec[c][t] = v;
            }
        }
        float fbar[CG][R];
#pragma unroll
        for (int c = 0; c < CG; ++c)
#pragma unroll
            for (int t = 0; t < R; ++t) fbar[c][t] = 0.0f;
        for (int l = 0; l < K; ++l) {
            float acc[R], cl[R], accd[R];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                acc[t] = 0.0f;
                accd[t] = 0.0f;
                cl[t] = (MODE == AM_GAMMA && act && y0 + t < a.H)
                            ? a.Cpl[(long long)l * a.Np + (long long)(y0 + t) * a.Wp + x]
                            : 0.0f;
            }
            // one copy of the plane loop (a uniform switch picks the
            // channel's registers: unrolled, the GAMMA pass took 264 VGPRs),
            // one LDS copy of a plane
            auto upd = [&](const float (&v)[R], float (&fb)[R], int gi, const float (&sv)[R],
                           const float (&sd)[R]) {
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    acc[t] = fmaf(v[t], sv[t], acc[t]);
                    if (MODE == AM_BETAS) accd[t] = fmaf(v[t], sd[t], accd[t]);
                    if (MODE == AM_GAMMA && gi > 0) fb[t] = fmaf(cl[t], sv[t], fb[t]);
                }
            };
            const int nch = min(CG, n + 1 - g * CG);
#pragma unroll 1
            for (int c = 0; c < nch; ++c) {
                int ng = g, nl = l, nc = c;
                const bool more = plane_next(n, K, ng, nl, nc);
                if (more) fetch(plane_index(n, ng, nl, nc), pre);
                const float* col = tbuf + ly0 * TXC + lx;
                float win[WIN];
#pragma unroll
                for (int q = 0; q < WIN; ++q) win[q] = col[q * TXC];
                float sv[R], sd[R];
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    float v = a.w[0] * win[t + S];
#pragma unroll
                    for (int j = 1; j <= S; ++j) v = fmaf(a.w[j], win[t + S - j] + win[t + S + j], v);
                    sv[t] = v;
                    float vd = 0.0f;  // wd[0] = 0
                    if (MODE == AM_BETAS) {
#pragma unroll
                        for (int j = 1; j <= S; ++j) vd = fmaf(a.wd[j], win[t + S - j] + win[t + S + j], vd);
                    }
                    sd[t] = vd;
                }
                switch (c) {
                    case 0: upd(vec[0], fbar[0], g * CG, sv, sd); break;
                    case 1: upd(vec[1], fbar[1], g * CG + 1, sv, sd); break;
                    case 2: upd(vec[2], fbar[2], g * CG + 2, sv, sd); break;
                    default: upd(vec[3], fbar[3], g * CG + 3, sv, sd); break;
                }
                __syncthreads();
                if (more) stash(tbuf, pre);
                __syncthreads();
            }
            if (act) {
                const long long off = (long long)l * a.Np + (long long)y0 * a.Wp + x;
                float* dst = (MODE == AM_GAMMA ? a.gamma : a.beta) + off;
                for (int t = 0; t < R && y0 + t < a.H; ++t) {
                    *dst = ((g == 0 && !a.bacc) ? 0.0f : *dst) + acc[t];
                    dst += a.Wp;
                }
                if (MODE == AM_BETAS) {
                    float* dd = a.betas + off;
                    for (int t = 0; t < R && y0 + t < a.H; ++t) {
                        *dd = (g == 0 ? 0.0f : *dd) + accd[t];
                        dd += a.Wp;
                    }
                }
            }
        }
        if (MODE == AM_GAMMA && act && a.gradf != nullptr) {
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                const int gi = g * CG + c;
                if (gi > n) break;
                if (gi == 0) continue;
                float* op = a.gradf + (long long)(gi - 1) * a.N + (long long)y0 * a.W + x;
                for (int t = 0; t < R && y0 + t < a.H; ++t) {
                    *op = fbar[c][t];
                    op += a.W;
                }
            }
        }
    }
}

template <int S, int MODE>
__global__ __launch_bounds__(RT) void col_adj(FA a) {
    col_adj_body<S, MODE>(a, (int)blockIdx.x);
}

template <int S, int MODE>
__global__ __launch_bounds__(RT) void col_adj_batch(const FA* __restrict__ fas, const int* __restrict__ pre,
                                                    int B) {
    int b;
    const int t = batch_block(pre, B, b);
    col_adj_body<S, MODE>(fas[b], t);
}

// Per-pixel end of the adjoint: dL/db = beta + A^+ gamma (A^+ symmetric),
// dL/dp = sum_l dL/db_l b_l (-2 s)(p - mu_l) with s = 1 / (2 sigma_r^2), and
// this pixel's share of dL/dsigma_r:
//   sum_l dL/db_l b_l |p - mu_l|^2 / sigma_r^3  +  gamma . (M b),
// M = d(A^+)/dsigma_r (K x K, formed on the host).  One launch covers the
// clusters l in [l0, l0 + 32) (dL/dp is linear in the per-cluster terms, so a
// second launch adds its share); the FP64 shares are summed per block in a
// fixed order.
constexpr int KF = 32;

__device__ __forceinline__ void adj_final_body(const FA& a, const float* __restrict__ Md, float sig3inv, int l0,
                                               int accumulate, float* __restrict__ gradp, double* part_slot,
                                               double* parts_slot, int blk) {
    // column m of the block's rows of A^+ and M, zero-padded to KF rows, so
    // the unrolled loops below carry no bounds branches
    __shared__ float sP[64 * KF], sA[64 * KF];
    __shared__ float smu[KF * FHD_MAX_RHO];
    __shared__ float sall[64 * 8];  // every center, dims padded to 8 (weights inline)
    __shared__ double red[RT / 64], reds[RT / 64];
    const int K = a.K, rho = a.rho;
    // without B planes (guides of at most 8 dimensions) b_m is recomputed
    // here exactly as the weights pass and the inline row pass form it
    const bool inl = a.Bpl == nullptr;
    const int kl = min(KF, K - l0);
    const int rp = rho <= 8 ? 8 : rho;  // center row pitch, zero-padded to 8 for short guides
    for (int t = threadIdx.x; t < K * KF; t += RT) {
        const int m = t / KF, l = t - m * KF;
        sP[t] = l < kl ? a.P[(long long)(l0 + l) * K + m] : 0.0f;
        sA[t] = l < kl ? Md[(long long)(l0 + l) * K + m] : 0.0f;
    }
    for (int t = threadIdx.x; t < KF * rp; t += RT) {
        const int l = t / rp, r = t - l * rp;
        smu[t] = (l < kl && r < rho) ? a.mu[(long long)(l0 + l) * rho + r] : 0.0f;
    }
    if (inl)
        for (int t = threadIdx.x; t < K * 8; t += RT) {
            const int m = t / 8, r = t - m * 8;
            sall[t] = r < rho ? a.mu[(long long)m * rho + r] : 0.0f;
        }
    __syncthreads();
    const long long i = (long long)blk * RT + threadIdx.x;
    const bool valid = i < a.N;
    const int y = valid ? (int)(i / a.W) : 0, x = valid ? (int)(i % a.W) : 0;
    const long long po = (long long)y * a.Wp + x;
    float pr8[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) pr8[r] = (valid && r < rho) ? a.p[(long long)r * a.N + i] : 0.0f;
    auto b_inline = [&](const float* mu8) {
        float d2 = 0.0f;
#pragma unroll
        for (int r = 0; r < 8; ++r) {  // padded entries: (0 - 0)^2
            const float d = pr8[r] - mu8[r];
            d2 = fmaf(d, d, d2);
        }
        return __expf(-d2 * a.inv2s2);
    };
    float pg[KF], ac[KF];
#pragma unroll
    for (int l = 0; l < KF; ++l) pg[l] = ac[l] = 0.0f;
    for (int m = 0; m < K; ++m) {
        const float gm = valid ? a.gamma[(long long)m * a.Np + po] : 0.0f;
        const float bm = !valid ? 0.0f : (inl ? b_inline(sall + m * 8) : a.Bpl[(long long)m * a.Np + po]);
        const float* cp = sP + m * KF;
        const float* ca = sA + m * KF;
#pragma unroll
        for (int l = 0; l < KF; ++l) {
            pg[l] = fmaf(cp[l], gm, pg[l]);
            ac[l] = fmaf(ca[l], bm, ac[l]);
        }
    }
    // weights w_l = dL/db_l * b_l (rows l >= kl of A^+ are zero, so pg[l] = 0 there)
    double sig = 0.0, sigs = 0.0;
    float wsum = 0.0f;
#pragma unroll
    for (int l = 0; l < KF; ++l) {
        if (l >= kl) break;
        const long long pl = (long long)(l0 + l) * a.Np + po;
        const float bl = !valid ? 0.0f : (inl ? b_inline(sall + (l0 + l) * 8) : a.Bpl[pl]);
        const float gl = valid ? a.gamma[pl] : 0.0f;
        const float bb = (valid ? a.beta[pl] : 0.0f) + pg[l];
        const float w = bb * bl;
        float d2 = 0.0f;
        if (rho <= 8) {
#pragma unroll
            for (int r = 0; r < 8; ++r) {  // padded entries: (0 - 0)^2
                const float d = pr8[r] - smu[l * rp + r];
                d2 = fmaf(d, d, d2);
            }
        } else {
            for (int r = 0; r < rho; ++r) {
                const float d = (valid ? a.p[(long long)r * a.N + i] : 0.0f) - smu[l * rp + r];
                d2 = fmaf(d, d, d2);
            }
        }
        sig += (double)w * d2 * sig3inv + (double)gl * ac[l];
        // dL/dsigma_s: b_l(i) Y(i) . ((d omega / d sigma_s) * (c_l [f, 1]))(i)
        if (a.betas != nullptr && valid) sigs += (double)bl * a.betas[pl];
        pg[l] = w;  // reuse: w_l
        wsum += w;
    }
    if (valid && gradp != nullptr) {
        const float m2s = -2.0f * a.inv2s2;
        for (int r = 0; r < rho; ++r) {
            float s = 0.0f;
#pragma unroll
            for (int l = 0; l < KF; ++l) s = fmaf(pg[l], smu[l * rp + r], s);
            const float pr = a.p[(long long)r * a.N + i];
            float* gp = gradp + (long long)r * a.N + i;
            const float v = m2s * (pr * wsum - s);
            *gp = accumulate ? *gp + v : v;
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        sig += __shfl_xor(sig, o, 64);
        sigs += __shfl_xor(sigs, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = sig;
        reds[threadIdx.x >> 6] = sigs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0, ts = 0.0;
        for (int q = 0; q < RT / 64; ++q) {
            t += red[q];
            ts += reds[q];
        }
        *part_slot = t;
        if (parts_slot != nullptr) *parts_slot = ts;
    }
}

__global__ __launch_bounds__(RT) void adj_final(FA a, const float* __restrict__ Md, float sig3inv, int l0,
                                                int accumulate, float* __restrict__ gradp,
                                                double* __restrict__ part, double* __restrict__ parts) {
    adj_final_body(a, Md, sig3inv, l0, accumulate, gradp, part + blockIdx.x,
                   parts != nullptr ? parts + blockIdx.x : nullptr, (int)blockIdx.x);
}

// The same end of the adjoint on the matrix cores, for short guides (rho <= 8,
// b recomputed inline) and K <= 32.  A wave takes 32 pixels at a time and
// forms the two K x K products of all of them as 16 steps each of the
// 32 x 32 x 2 FP32 matrix product:
//   C1[l][j] = sum_m A^+[l][m] gamma_m(j),   C2[l][j] = sum_m M[l][m] gamma_m(j)
// (lane t supplies A^+[t % 32][2s + t / 32] and M[...] from registers loaded
// once per block, and gamma_{2s + t / 32} of pixel t % 32; the matrices are
// zero-padded to 32).  Lane t then holds both products for pixel t % 32 and
// the 16 clusters l = 8 (r / 4) + 4 (t / 32) + r % 4, r < 16, and finishes
// those (pixel, cluster) pairs in place, loading beta_l (consecutive lanes:
// consecutive pixels of one plane):
//   dL/db_l = beta_l + C1[l],  w_l = dL/db_l b_l,
//   share of dL/dsigma_r = sum_l w_l |p - mu_l|^2 / sigma_r^3 + b_l C2[l]
// (M symmetric: gamma . (M b) = b . (M gamma)), and dL/dp from sum_l w_l and
// sum_l w_l mu_l, the two lanes of a pixel added by a swap across the wave
// halves.  FP64 shares: per lane in pixel-group order, then the fixed shuffle
// tree and wave order.
constexpr int AF_GROUPS = 8;              // 32-pixel groups per wave
constexpr int AF_PIX = RT / 2 * AF_GROUPS; // pixels per block

// 32-bit byte offsets from a uniform base (the planes of one image span less
// than 4 GiB where this is used): one register per address, and the load
// takes the scalar base directly
__device__ __forceinline__ float ld_off(const float* base, unsigned byte_off) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <int RH>
__device__ __forceinline__ void adj_final_mfma_rh(const FA& a, const float* __restrict__ Md, float sig3inv,
                                                    float* __restrict__ gradp, double* part_slot,
                                                    double* parts_slot, int blk) {
    __shared__ float smu[KMAX_INLINE * RHO_INLINE];
    __shared__ double red[RT / 64], reds[RT / 64];
    const int K = a.K, rho = a.rho;
    for (int t = threadIdx.x; t < KMAX_INLINE * RHO_INLINE; t += RT) {
        const int l = t / RHO_INLINE, r = t - l * RHO_INLINE;
        smu[t] = (l < K && r < rho) ? a.mu[l * rho + r] : 0.0f;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int jl = lane & 31, kh = lane >> 5;
    // A operands: A^+[jl][2s + kh] and M[jl][2s + kh]
    float Pa[16], Ma[16];
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
        const int m = 2 * s2 + kh;
        const bool in = jl < K && m < K;
        Pa[s2] = in ? a.P[jl * K + m] : 0.0f;
        Ma[s2] = in ? Md[jl * K + m] : 0.0f;
    }
    __syncthreads();
    const float m2s = -2.0f * a.inv2s2;
    const unsigned np4 = (unsigned)a.Np * 4u, n4 = (unsigned)a.N * 4u;
    double sig = 0.0, sigs = 0.0;
#pragma unroll 1
    for (int grp = 0; grp < AF_GROUPS; ++grp) {
        // an offset the compiler cannot see through keeps the centers as LDS
        // reads inside the loop (hoisted out of it they take 128 registers)
        int lo = 0;
        asm volatile("" : "+v"(lo));
        const float* smq = smu + lo;
        const long long i = ((long long)blk * (RT / 64) + wave) * (32LL * AF_GROUPS) + grp * 32 + jl;
        const bool valid = i < a.N;
        const int ii = valid ? (int)i : 0;  // loads stay in bounds; invalid lanes are zeroed after
        const int y = ii / a.W, x = ii - y * a.W;
        const unsigned po4 = (unsigned)(y * a.Wp + x) * 4u, pi4 = (unsigned)ii * 4u;
        // running offsets, clamped to the last plane (the value is zeroed there)
        const unsigned last = po4 + (unsigned)(K - 1) * np4;
        float gv[16];
        unsigned og = po4 + (unsigned)kh * np4;
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) {
            const int m = 2 * s2 + kh;
            const float v = ld_off(a.gamma, min(og, last));
            gv[s2] = (valid && m < K) ? v : 0.0f;
            og += 2u * np4;
        }
        float pr[RH];
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            const float v = ld_off(a.p, pi4 + (unsigned)min(r, rho - 1) * n4);
            pr[r] = (valid && r < rho) ? v : 0.0f;
        }
        f32x16 c1, c2;
#pragma unroll
        for (int r = 0; r < 16; ++r) c1[r] = c2[r] = 0.0f;
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) {
            c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(Pa[s2], gv[s2], c1, 0, 0, 0);
            c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(Ma[s2], gv[s2], c2, 0, 0, 0);
        }
        float bt[16], bs[16];
        unsigned ob = po4 + 4u * (unsigned)kh * np4;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int l = 8 * (r >> 2) + 4 * kh + (r & 3);
            const unsigned off = min(ob, last);
            ob += ((r & 3) == 3 ? 5u : 1u) * np4;  // l runs 4 kh + 0..3, then 8 on
            const float v = ld_off(a.beta, off);
            bt[r] = (valid && l < K) ? v : 0.0f;
            bs[r] = 0.0f;
            if (a.betas != nullptr) {
                const float vs = ld_off(a.betas, off);
                bs[r] = (valid && l < K) ? vs : 0.0f;
            }
        }
        float wsum = 0.0f, sw[RH];
#pragma unroll
        for (int r = 0; r < RH; ++r) sw[r] = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int l = 8 * (r >> 2) + 4 * kh + (r & 3);
            float mu8[RH];
#pragma unroll
            for (int q = 0; q < RH; ++q) mu8[q] = smq[l * RHO_INLINE + q];
            float d2 = 0.0f;
#pragma unroll
            for (int q = 0; q < RH; ++q) {  // padded entries: (0 - 0)^2
                const float d = pr[q] - mu8[q];
                d2 = fmaf(d, d, d2);
            }
            // b_l exactly as the weights pass and the inline row pass form it
            const float bl = (valid && l < K) ? __expf(-d2 * a.inv2s2) : 0.0f;
            const float w = (bt[r] + c1[r]) * bl;
            sig += (double)w * d2 * sig3inv + (double)bl * c2[r];
            sigs += (double)bl * bs[r];
            wsum += w;
#pragma unroll
            for (int q = 0; q < RH; ++q) sw[q] = fmaf(w, mu8[q], sw[q]);
        }
        // the pixel's other 16 clusters sit in the lane 32 apart
        wsum += __shfl_xor(wsum, 32, 64);
#pragma unroll
        for (int q = 0; q < RH; ++q) sw[q] += __shfl_xor(sw[q], 32, 64);
        if (valid && kh == 0 && gradp != nullptr) {
#pragma unroll
            for (int q = 0; q < RH; ++q)
                if (q < rho) gradp[(long long)q * a.N + ii] = m2s * (pr[q] * wsum - sw[q]);
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        sig += __shfl_xor(sig, o, 64);
        sigs += __shfl_xor(sigs, o, 64);
    }
    if (lane == 0) {
        red[wave] = sig;
        reds[wave] = sigs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0, ts = 0.0;
        for (int q = 0; q < RT / 64; ++q) {
            t += red[q];
            ts += reds[q];
        }
        *part_slot = t;
        if (parts_slot != nullptr) *parts_slot = ts;
    }
}

// RH: guide dimensions summed per distance (4 for guides of at most 4
// dimensions: the entries past rho are zero on both sides).
__device__ __forceinline__ void adj_final_mfma_body(const FA& a, const float* __restrict__ Md, float sig3inv,
                                                    float* __restrict__ gradp, double* part_slot,
                                                    double* parts_slot, int blk) {
    if (a.rho <= 4)
        adj_final_mfma_rh<4>(a, Md, sig3inv, gradp, part_slot, parts_slot, blk);
    else
        adj_final_mfma_rh<RHO_INLINE>(a, Md, sig3inv, gradp, part_slot, parts_slot, blk);
}

__global__ __launch_bounds__(RT) void adj_final_mfma(FA a, const float* __restrict__ Md, float sig3inv,
                                                     float* __restrict__ gradp, double* __restrict__ part,
                                                     double* __restrict__ parts) {
    adj_final_mfma_body(a, Md, sig3inv, gradp, part + blockIdx.x, parts != nullptr ? parts + blockIdx.x : nullptr,
                        (int)blockIdx.x);
}

__global__ __launch_bounds__(RT) void adj_final_mfma_batch(const FA* __restrict__ fas, const int* __restrict__ pre,
                                                           int B, float sig3inv, double* __restrict__ part) {
    int b;
    const int t = batch_block(pre, B, b);
    const FA& a = fas[b];
    adj_final_mfma_body(a, a.Md, sig3inv, a.gradp, part + blockIdx.x, nullptr, t);
}

__global__ __launch_bounds__(RT) void sum_blocks(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double red[RT / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += RT) s += part[b];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < RT / 64; ++q) t += red[q];
        *out = t;
    }
}

// ---------------------------------------------------------------------------
// Recursive Gaussian window (Young and van Vliet; the paper's O(1) choice):
// every 1-D pass is the causal recursion w[t] = B u[t] + a1 w[t-1] +
// a2 w[t-2] + a3 w[t-3] from a zero state at the start, then the same
// anti-causal recursion from a zero state at the end.  Rows first (the
// factor c_l or b_l times [f, 1] formed on the fly from the materialised
// planes, rows walked in LDS tiles), then columns in place (one thread per
// plane column, adjacent threads on adjacent columns), then the
// recombination of eqs. (15)-(16) per pixel.  The planes have no halo rows
// (S = 0).
// Row recursions: a block of YT threads takes YT rows of one plane and walks
// them in YT x YT tiles staged in LDS (loaded and stored row-contiguously,
// so the global accesses coalesce); thread t runs the recursion of row t
// across each tile (pitch YT + 1: conflict-free in both directions).  A
// thread's YT loads of a tile column are issued together into registers
// (addresses clamped into the plane, values outside it zero) before they
// go to LDS, so they are in flight at once.
constexpr int YT = 64;

__global__ __launch_bounds__(YT) void row_young(FA a, const float* __restrict__ fac) {
    __shared__ float tile[YT][YT + 1];
    const int nyb = (a.H + YT - 1) / YT;
    const int pl = blockIdx.x / nyb, y0 = (blockIdx.x - pl * nyb) * YT;
    const int l = pl / (a.n + 1), ch = pl - l * (a.n + 1);
    const float* __restrict__ cb = fac + (long long)l * a.Np;
    const float* __restrict__ fb = ch < a.n ? a.f + (long long)ch * a.N : nullptr;
    float* __restrict__ db = a.planes + (long long)pl * a.Pp;
    const int t = threadIdx.x;
    const float B = a.yc[0], a1 = a.yc[1], a2 = a.yc[2], a3 = a.yc[3];
    float v[YT];
    // tile column x of rows y0 .. y0 + YT - 1 into v (zero outside the plane)
    auto load_col = [&](const float* __restrict__ src, long long pitch, const float* __restrict__ mul, int x) {
        const int xc = min(x, a.W - 1);
#pragma unroll
        for (int r = 0; r < YT; ++r) {
            const int yc = min(y0 + r, a.H - 1);
            v[r] = src[(long long)yc * pitch + xc];
        }
        if (mul != nullptr) {
            float m[YT];
#pragma unroll
            for (int r = 0; r < YT; ++r) m[r] = mul[(long long)min(y0 + r, a.H - 1) * a.W + xc];
#pragma unroll
            for (int r = 0; r < YT; ++r) v[r] *= m[r];
        }
#pragma unroll
        for (int r = 0; r < YT; ++r) tile[r][t] = (y0 + r < a.H && x < a.W) ? v[r] : 0.0f;
    };
    auto store_col = [&](int x) {
#pragma unroll
        for (int r = 0; r < YT; ++r) v[r] = tile[r][t];
        if (x < a.W)
#pragma unroll
            for (int r = 0; r < YT; ++r)
                if (y0 + r < a.H) db[(long long)(y0 + r) * a.Wp + x] = v[r];
    };
    float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
    for (int x0 = 0; x0 < a.W; x0 += YT) {
        const int cnt = min(YT, a.W - x0);
        load_col(cb, a.Wp, fb, x0 + t);
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {  // causal: row t
            const float w = B * tile[t][k] + a1 * p1 + a2 * p2 + a3 * p3;
            tile[t][k] = w;
            p3 = p2;
            p2 = p1;
            p1 = w;
        }
        __syncthreads();
        store_col(x0 + t);
        __syncthreads();
    }
    p1 = p2 = p3 = 0.0f;
    for (int x0 = (a.W - 1) / YT * YT; x0 >= 0; x0 -= YT) {
        const int cnt = min(YT, a.W - x0);
        load_col(db, a.Wp, nullptr, x0 + t);
        __syncthreads();
        for (int k = cnt - 1; k >= 0; --k) {  // anti-causal: row t
            const float w = B * tile[t][k] + a1 * p1 + a2 * p2 + a3 * p3;
            tile[t][k] = w;
            p3 = p2;
            p2 = p1;
            p1 = w;
        }
        __syncthreads();
        store_col(x0 + t);
        __syncthreads();
    }
}

// Column recursions in place: one thread per plane column (adjacent threads
// on adjacent columns), YC elements of the column loaded together into
// registers per chunk (row indices clamped into the plane; elements past the
// end only advance a state that is then dropped, and are not stored).
constexpr int YC = 16;

__global__ __launch_bounds__(RT) void col_young(FA a) {
    const long long t = (long long)blockIdx.x * RT + threadIdx.x;
    const int planes = a.K * (a.n + 1);
    if (t >= (long long)planes * a.W) return;
    const int x = (int)(t % a.W);
    const int pl = (int)(t / a.W);
    float* __restrict__ col = a.planes + (long long)pl * a.Pp + x;
    const float B = a.yc[0], a1 = a.yc[1], a2 = a.yc[2], a3 = a.yc[3];
    const int H = a.H;
    float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
    for (int y0 = 0; y0 < H; y0 += YC) {
        float v[YC];
#pragma unroll
        for (int k = 0; k < YC; ++k) v[k] = col[(long long)min(y0 + k, H - 1) * a.Wp];
#pragma unroll
        for (int k = 0; k < YC; ++k) {
            const float w = B * v[k] + a1 * p1 + a2 * p2 + a3 * p3;
            v[k] = w;
            p3 = p2;
            p2 = p1;
            p1 = w;
        }
#pragma unroll
        for (int k = 0; k < YC; ++k)
            if (y0 + k < H) col[(long long)(y0 + k) * a.Wp] = v[k];
    }
    p1 = p2 = p3 = 0.0f;
    for (int y1 = H - 1; y1 >= 0; y1 -= YC) {  // rows y1, y1 - 1, ..., y1 - YC + 1
        float v[YC];
#pragma unroll
        for (int k = 0; k < YC; ++k) v[k] = col[(long long)max(y1 - k, 0) * a.Wp];
#pragma unroll
        for (int k = 0; k < YC; ++k) {
            const float w = B * v[k] + a1 * p1 + a2 * p2 + a3 * p3;
            v[k] = w;
            p3 = p2;
            p2 = p1;
            p1 = w;
        }
#pragma unroll
        for (int k = 0; k < YC; ++k)
            if (y1 - k >= 0) col[(long long)(y1 - k) * a.Wp] = v[k];
    }
}

// out = sum_l h_l V_l[0:n] / sum_l h_l V_l[n] with h_l = b_l(i) (least
// squares, transposed form) or the cluster indicator (hard variant)
__global__ __launch_bounds__(RT) void recomb_young(FA a, int hard) {
    const long long i = (long long)blockIdx.x * RT + threadIdx.x;
    if (i >= a.N) return;
    const long long po = (i / a.W) * a.Wp + i % a.W;
    const int n = a.n;
    const int lab = hard ? a.labels[i] : -1;
    auto h = [&](int l) { return hard ? (l == lab ? 1.0f : 0.0f) : a.Bpl[(long long)l * a.Np + po]; };
    float r = 0.0f;
    for (int l = 0; l < a.K; ++l) r = fmaf(h(l), a.planes[(long long)(l * (n + 1) + n) * a.Pp + po], r);
    if (a.den != nullptr) a.den[i] = r;
    const float inv = 1.0f / r;
    for (int ch = 0; ch < n; ++ch) {
        float v = 0.0f;
        for (int l = 0; l < a.K; ++l) v = fmaf(h(l), a.planes[(long long)(l * (n + 1) + ch) * a.Pp + po], v);
        a.out[(long long)ch * a.N + i] = v * inv;
    }
}

// ---------------------------------------------------------------------------
// Pixel sums for dL/dmu (centers gradient, assignment frozen):
//   Gm[l][m] = sum_i gamma_l(i) b_m(i)       (= dL/dA^+, since c = A^+ b)
//   S1[l]    = sum_i w_l(i),  S2[l][r] = sum_i w_l(i) p_r(i),
// w_l = dL/db_l b_l = (beta_l + (A^+ gamma)_l) b_l.  A fixed grid of blocks
// of one wave; each takes chunks of CMU pixels in turn: one thread per pixel
// forms b, gamma and w into LDS (row pitch CMU + 1, conflict-free), then one
// thread per sum entry adds the chunk's terms (FP64).  Each block writes its FP64 totals; sum_entries adds the
// blocks in order.
constexpr int CMU = 64;
constexpr int CMP = CMU + 1;
constexpr int MU_GRID = 1024;

size_t adj_centers_lds(int K, int rho) {
    const size_t E = (size_t)K * K + K + (size_t)K * rho;
    return sizeof(double) * E + sizeof(float) * ((size_t)K * K + (size_t)K * rho + 3 * (size_t)K * CMP +
                                                 (size_t)rho * CMP);
}

__global__ __launch_bounds__(CMU) void adj_centers(FA a, double* __restrict__ part) {
    extern __shared__ double smem[];
    const int K = a.K, rho = a.rho;
    const int E = K * K + K + K * rho;
    double* sacc = smem;
    float* sP = reinterpret_cast<float*>(sacc + E);  // A^+ (K x K)
    float* smu = sP + K * K;                          // centers (K x rho)
    float* sb = smu + K * rho;                        // b_m of the chunk's pixels
    float* sg = sb + K * CMP;                         // gamma_m
    float* sw = sg + K * CMP;                         // w_l
    float* spp = sw + K * CMP;                        // p_r
    const int t = threadIdx.x;
    for (int e = t; e < E; e += CMU) sacc[e] = 0.0;
    for (int e = t; e < K * K; e += CMU) sP[e] = a.P[e];
    for (int e = t; e < K * rho; e += CMU) smu[e] = a.mu[e];
    __syncthreads();
    const long long nch = (a.N + CMU - 1) / CMU;
    for (long long ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const long long i = ch * CMU + t;
        const bool valid = i < a.N;
        const long long po = valid ? (i / a.W) * a.Wp + i % a.W : 0;
        for (int r = 0; r < rho; ++r) spp[r * CMP + t] = valid ? a.p[(long long)r * a.N + i] : 0.0f;
        for (int m = 0; m < K; ++m) {
            float d2 = 0.0f;
            for (int r = 0; r < rho; ++r) {
                const float d = spp[r * CMP + t] - smu[m * rho + r];
                d2 = fmaf(d, d, d2);
            }
            sb[m * CMP + t] = valid ? __expf(-d2 * a.inv2s2) : 0.0f;
            sg[m * CMP + t] = valid ? a.gamma[(long long)m * a.Np + po] : 0.0f;
        }
        for (int l = 0; l < K; ++l) {
            float pg = 0.0f;
            for (int m = 0; m < K; ++m) pg = fmaf(sP[l * K + m], sg[m * CMP + t], pg);
            const float bt = valid ? a.beta[(long long)l * a.Np + po] : 0.0f;
            sw[l * CMP + t] = (bt + pg) * sb[l * CMP + t];
        }
        __syncthreads();
        // FP64 sums of the (exact) products of FP32 values: the pseudo-inverse
        // derivative amplifies rounding in these sums by up to 1 / lambda_min^2
        for (int e = t; e < E; e += CMU) {
            double s = 0.0;
            if (e < K * K) {
                const float* gl = sg + (e / K) * CMP;
                const float* bm = sb + (e % K) * CMP;
                for (int q = 0; q < CMU; ++q) s = fma((double)gl[q], (double)bm[q], s);
            } else if (e < K * K + K) {
                const float* wl = sw + (e - K * K) * CMP;
                for (int q = 0; q < CMU; ++q) s += (double)wl[q];
            } else {
                const int f = e - K * K - K;
                const float* wl = sw + (f / rho) * CMP;
                const float* pr = spp + (f % rho) * CMP;
                for (int q = 0; q < CMU; ++q) s = fma((double)wl[q], (double)pr[q], s);
            }
            sacc[e] += s;
        }
        __syncthreads();
    }
    for (int e = t; e < E; e += CMU) part[(long long)blockIdx.x * E + e] = sacc[e];
}

// out[e] = sum over b < nb of part[b * E + e], in order
__global__ __launch_bounds__(RT) void sum_entries(const double* __restrict__ part, int nb, int E,
                                                  double* __restrict__ out) {
    const int e = blockIdx.x * RT + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(long long)b * E + e];
    out[e] = s;
}

// ---------------------------------------------------------------------------
// Weights pass (guides with more than RHO_INLINE dimensions, more than
// KMAX_INLINE clusters, or the adjoint): B and C planes.  One thread per pixel
// of a row run of blockDim.x pixels.  Centers (rho padded to a multiple of 8)
// and A^+ (columns padded to a multiple of 8) sit in LDS with zero padding, so
// the loops carry no bounds branches: padded dimensions add (0 - 0)^2 and
// padded columns produce coefficients that are never stored.
__host__ __device__ constexpr int pad8(int v) { return (v + 7) & ~7; }

size_t weights_fp32_lds(int K, int rho, int npx) {
    return sizeof(float) * ((size_t)K * pad8(K) + (size_t)K * pad8(rho) + (size_t)K * npx);
}

int weights_fp32_npx(int K) { return K <= 64 ? RT : 64; }

__device__ __forceinline__ void weights_fp32_body(const FA& a, float* Bpl, float* Cpl, int bx, int by) {
    extern __shared__ float lds[];
    const int K = a.K, rho = a.rho, KP = pad8(K), RP = pad8(rho);
    const int npx = blockDim.x;
    float* sP = lds;              // K x KP
    float* smu = sP + K * KP;     // K x RP
    float* bs = smu + K * RP;     // K x npx (center-major)
    for (int t = threadIdx.x; t < K * KP; t += npx) {
        const int m = t / KP, l = t - m * KP;
        sP[t] = l < K ? a.P[m * K + l] : 0.0f;
    }
    for (int t = threadIdx.x; t < K * RP; t += npx) {
        const int m = t / RP, r = t - m * RP;
        smu[t] = r < rho ? a.mu[m * rho + r] : 0.0f;
    }
    __syncthreads();
    const int y = by, x = bx * npx + threadIdx.x;
    if (x >= a.W) return;
    const long long pix = (long long)y * a.W + x;
    const long long ppl = (long long)y * a.Wp + x;
    for (int m = 0; m < K; ++m) bs[m * npx + threadIdx.x] = 0.0f;
    for (int r0 = 0; r0 < RP; r0 += 8) {
        float pr[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) pr[r] = r0 + r < rho ? a.p[(long long)(r0 + r) * a.N + pix] : 0.0f;
        for (int m = 0; m < K; ++m) {
            const float* mu = smu + m * RP + r0;
            float d2 = bs[m * npx + threadIdx.x];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const float d = pr[r] - mu[r];
                d2 = fmaf(d, d, d2);
            }
            bs[m * npx + threadIdx.x] = d2;
        }
    }
    for (int m = 0; m < K; ++m) {
        const float b = __expf(-bs[m * npx + threadIdx.x] * a.inv2s2);
        bs[m * npx + threadIdx.x] = b;
        if (Bpl != nullptr) Bpl[(long long)m * a.Np + ppl] = b;
    }
    if (Cpl == nullptr) return;
    for (int l0 = 0; l0 < K; l0 += 8) {
        float acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
        for (int m = 0; m < K; ++m) {
            const float bv = bs[m * npx + threadIdx.x];
            const float* prow = sP + m * KP + l0;  // A^+ symmetric: row m = column m
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = fmaf(prow[q], bv, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (l0 + q < K) Cpl[(long long)(l0 + q) * a.Np + ppl] = acc[q];
    }
}

__global__ __launch_bounds__(RT) void weights_fp32(FA a, float* Bpl, float* Cpl) {
    weights_fp32_body(a, Bpl, Cpl, (int)blockIdx.x, (int)blockIdx.y);
}

// batched adjoint (weights inline elsewhere): the C planes of every image
__global__ __launch_bounds__(RT) void weights_fp32_batch(const FA* __restrict__ fas, const int* __restrict__ pre,
                                                         int B) {
    int b;
    const int t = batch_block(pre, B, b);
    const FA& a = fas[b];
    const int gx = (a.W + (int)blockDim.x - 1) / (int)blockDim.x;
    weights_fp32_body(a, nullptr, const_cast<float*>(a.Cpl), t % gx, t / gx);
}

// ---------------------------------------------------------------------------
// Weights pass with the point-to-center distance as a matrix contraction on
// the matrix cores: D = |p~|^2 + |mu~|^2 - 2 p~ . mu~, where p~ = round(p - o)
// and mu~ = round(mu - o) are BF16 or FP16 values (o is the mean of the
// centers: distances do not change under a common shift, and the shift keeps
// the rounded coordinates small).  Products of 16-bit values are exact in the
// FP32 accumulator, and the norms are taken from the same rounded values, so
// D is the distance between the rounded points up to FP32 accumulation; it is
// clamped at 0.  b = exp(-D / 2 sigma_r^2) in FP32, c = A^+ b in FP32.
// A block handles 64 pixels of a row, each wave 16 of them against all
// centers, 16 centers per 16x16x16 product (dims in chunks of 16).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

constexpr int MW_PIX = 64;                      // pixels per block
constexpr int MW_RHO = FHD_MAX_RHO;             // padded dims
constexpr int MW_K = FHD_MAX_K;

__device__ __forceinline__ unsigned short to_bf16(float x) {
    // round to nearest even (finite inputs)
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <bool BF16>
__device__ __forceinline__ unsigned short round16(float x) {
    if (BF16) return to_bf16(x);
    const _Float16 h = (_Float16)x;
    return *reinterpret_cast<const unsigned short*>(&h);
}
template <bool BF16>
__device__ __forceinline__ float widen16(unsigned short v) {
    if (BF16) return from_bf16(v);
    return (float)*reinterpret_cast<const _Float16*>(&v);
}

template <bool BF16>
__global__ __launch_bounds__(RT) void weights_mfma(FA a, float* Bpl, float* Cpl, const float* offs) {
    __shared__ unsigned short smu[MW_K * MW_RHO];  // rounded centers, dims padded with 0
    __shared__ float smn[MW_K];                    // |mu~|^2
    __shared__ float spn[MW_PIX];                  // |p~|^2
    __shared__ float sb[MW_PIX * (MW_K + 1)];      // b for the block's pixels
    extern __shared__ float sPp[];                 // A^+, K x pad8(K), zero-padded columns
    const int K = a.K, rho = a.rho, KP = pad8(K);
    const int rp = (rho + 15) & ~15;               // dims rounded up to whole chunks
    const int y = blockIdx.y, x0 = blockIdx.x * MW_PIX;
    for (int t = threadIdx.x; t < K * rp; t += RT) {
        const int k = t / rp, d = t - k * rp;
        smu[k * MW_RHO + d] = d < rho ? round16<BF16>(a.mu[k * rho + d] - offs[d]) : (unsigned short)0;
    }
    if (Cpl != nullptr)
        for (int t = threadIdx.x; t < K * KP; t += RT) {
            const int m = t / KP, l = t - m * KP;
            sPp[t] = l < K ? a.P[m * K + l] : 0.0f;
        }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += RT) {
        float s = 0.0f;
        for (int d = 0; d < rho; ++d) {
            const float v = widen16<BF16>(smu[k * MW_RHO + d]);
            s = fmaf(v, v, s);
        }
        smn[k] = s;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;       // fragment row / dim quad
    const int pix = wave * 16 + i;                 // this lane's pixel for the A fragment
    const int x = x0 + pix;
    const bool inx = x < a.W;
    const long long off = (long long)y * a.W + x;
    // A fragments: pixel pix, dims 16c + 4kq + e
    unsigned short af[MW_RHO / 4];
    float pn = 0.0f;
#pragma unroll
    for (int c = 0; c < MW_RHO / 16; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int d = 16 * c + 4 * kq + e;
            unsigned short v = 0;
            if (16 * c < rp && d < rho && inx) v = round16<BF16>(a.p[(long long)d * a.N + off] - offs[d]);
            af[4 * c + e] = v;
            const float w = widen16<BF16>(v);
            pn = fmaf(w, w, pn);
        }
    pn += __shfl_xor(pn, 16, 64);
    pn += __shfl_xor(pn, 32, 64);
    if (kq == 0) spn[pix] = pn;
    __syncthreads();
    for (int t0 = 0; t0 < K; t0 += 16) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        const int cen = t0 + i;                    // B fragment column (center)
#pragma unroll
        for (int c = 0; c < MW_RHO / 16; ++c) {
            if (16 * c >= rp) break;
            i16x4 av, bv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                av[e] = (short)af[4 * c + e];
                bv[e] = cen < K ? (short)smu[cen * MW_RHO + 16 * c + 4 * kq + e] : (short)0;
            }
            if (BF16) {
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
            } else {
                acc = __builtin_amdgcn_mfma_f32_16x16x16f16(*reinterpret_cast<f16x4*>(&av),
                                                            *reinterpret_cast<f16x4*>(&bv), acc, 0, 0, 0);
            }
        }
        // acc[e] = p~(pixel wave*16 + 4kq + e) . mu~(center t0 + i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int pr = wave * 16 + 4 * kq + e;
            if (cen < K) {
                const float d2 = fmaxf(spn[pr] + smn[cen] - 2.0f * acc[e], 0.0f);
                sb[pr * (MW_K + 1) + cen] = __expf(-d2 * a.inv2s2);
            }
        }
    }
    __syncthreads();
    const long long prow = (long long)y * a.Wp;
    for (int t = threadIdx.x; t < MW_PIX * K; t += RT) {
        const int l = t / MW_PIX, h = t - l * MW_PIX;
        if (x0 + h < a.W) Bpl[(long long)l * a.Np + prow + x0 + h] = sb[h * (MW_K + 1) + l];
    }
    if (Cpl == nullptr) return;
    const int groups = (K + 7) >> 3;
    for (int t = threadIdx.x; t < MW_PIX * groups; t += RT) {
        const int g = t / MW_PIX, h = t - g * MW_PIX;
        if (x0 + h >= a.W) continue;
        float acc2[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc2[q] = 0.0f;
        for (int m = 0; m < K; ++m) {
            const float bv = sb[h * (MW_K + 1) + m];
            const float* prow2 = sPp + m * KP + g * 8;  // A^+ symmetric: row m = column m
#pragma unroll
            for (int q = 0; q < 8; ++q) acc2[q] = fmaf(prow2[q], bv, acc2[q]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (g * 8 + q < K) Cpl[(long long)(g * 8 + q) * a.Np + prow + x0 + h] = acc2[q];
    }
}

// ---------------------------------------------------------------------------
// Brute force, eqs. (1)-(2), in FP32: each thread takes one column and R
// consecutive output rows.  For each horizontal offset jx it walks the R + 2S
// neighbour rows of its column once, loading each neighbour's guide (and
// image) values once for all of its R outputs whose window holds that
// neighbour; the sums stay in registers.  A wave's 64 lanes take 64
// consecutive columns (coalesced loads, served by the caches across
// offsets), the block's four waves consecutive groups of R rows.  RM, NM
// bound the guide and image channels (EXACT: exactly RM, NM); SAME: the
// image is the guide (one load serves both); beyond 32 channels (DIRECT)
// the values are read per use instead of staged in registers.
template <int R, int RM, int NM, bool EXACT, bool SAME>
__global__ __launch_bounds__(RT) void brute_strip(FA a) {
    constexpr bool DIRECT = RM > 32 || NM > 32;
    constexpr int RS = DIRECT ? 1 : RM, NS = DIRECT || SAME ? 1 : NM;
    const int S = a.S;
    const int rho = EXACT ? RM : a.rho, n = EXACT ? NM : a.n;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y0 = (blockIdx.y * (RT / 64) + (threadIdx.x >> 6)) * R;  // uniform per wave
    if (y0 >= a.H) return;
    const bool colin = x < a.W;
    const int xc = colin ? x : a.W - 1;  // out-of-image lanes read a valid column and store nothing
    float pc[R][RM], num[R][NM], eta[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long off = (long long)min(y0 + r, a.H - 1) * a.W + xc;
#pragma unroll
        for (int c = 0; c < RM; ++c) pc[r][c] = c < rho ? a.p[(long long)c * a.N + off] : 0.0f;
#pragma unroll
        for (int c = 0; c < NM; ++c) num[r][c] = 0.0f;
        eta[r] = 0.0f;
    }
    // neighbour rows y0 - S + t inside the image
    const int t0 = max(0, S - y0), t1 = min(R + 2 * S, a.H - y0 + S);
    for (int jx = -S; jx <= S; ++jx) {
        const int xx = xc - jx;
        const bool inx = colin && xx >= 0 && xx < a.W;
        const int xq = min(max(xx, 0), a.W - 1);
        const float wx = a.w[jx < 0 ? -jx : jx];
        for (int t = t0; t < t1; ++t) {
            const long long q = (long long)(y0 - S + t) * a.W + xq;
            float pq[RS], fq[NS];
            if (!DIRECT) {
#pragma unroll
                for (int c = 0; c < RS; ++c) pq[c] = c < rho ? a.p[(long long)c * a.N + q] : 0.0f;
                if (!SAME) {
#pragma unroll
                    for (int c = 0; c < NS; ++c) fq[c] = c < n ? a.f[(long long)c * a.N + q] : 0.0f;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int jy = r + S - t;  // output row y0 + r minus the neighbour row
                if (jy < -S || jy > S) continue;  // uniform
                float d2 = 0.0f;
#pragma unroll
                for (int c = 0; c < RM; ++c) {
                    if (c < rho) {
                        const float v = DIRECT ? a.p[(long long)c * a.N + q] : pq[DIRECT ? 0 : c];
                        const float d = v - pc[r][c];
                        d2 = fmaf(d, d, d2);
                    }
                }
                const float wgt = inx ? wx * a.w[jy < 0 ? -jy : jy] * __expf(-d2 * a.inv2s2) : 0.0f;
#pragma unroll
                for (int c = 0; c < NM; ++c) {
                    if (c < n) {
                        const float v = DIRECT ? a.f[(long long)c * a.N + q]
                                               : (SAME ? pq[c < RS ? c : 0] : fq[c < NS ? c : 0]);
                        num[r][c] = fmaf(wgt, v, num[r][c]);
                    }
                }
                eta[r] += wgt;
            }
        }
    }
    if (!colin) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (y0 + r >= a.H) break;
        const long long off = (long long)(y0 + r) * a.W + x;
        const float inv = 1.0f / eta[r];
#pragma unroll
        for (int c = 0; c < NM; ++c)
            if (c < n) a.out[(long long)c * a.N + off] = num[r][c] * inv;
        if (a.den) a.den[off] = eta[r];
    }
}

// ---------------------------------------------------------------------------
// dispatch tables for the unrolled radii

using KernFn = void (*)(FA);

template <int S>
struct Tables {
    static void fill(KernFn* row, KernFn (*col)[3]) {
        row[S] = row_gauss<S>;
        col[S][WM_INLINE] = col_gauss<S, WM_INLINE>;
        col[S][WM_PLANES] = col_gauss<S, WM_PLANES>;
        col[S][WM_HARD] = col_gauss<S, WM_HARD>;
        Tables<S - 1>::fill(row, col);
    }
};
template <>
struct Tables<0> {
    static void fill(KernFn*, KernFn (*)[3]) {}
};

typedef void (*BatchFn)(const FA*, const int*, int);
template <int S>
struct BatchTables {
    static void fill(BatchFn* row, BatchFn (*col)[3]) {
        row[S] = row_gauss_batch<S>;
        col[S][WM_INLINE] = col_gauss_batch<S, WM_INLINE>;
        col[S][WM_PLANES] = col_gauss_batch<S, WM_PLANES>;
        col[S][WM_HARD] = col_gauss_batch<S, WM_HARD>;
        BatchTables<S - 1>::fill(row, col);
    }
};
template <>
struct BatchTables<0> {
    static void fill(BatchFn*, BatchFn (*)[3]) {}
};

template <int S>
struct AdjTables {
    static void fill(KernFn (*adj)[3]) {
        adj[S][AM_BETA] = col_adj<S, AM_BETA>;
        adj[S][AM_GAMMA] = col_adj<S, AM_GAMMA>;
        adj[S][AM_BETAS] = col_adj<S, AM_BETAS>;
        AdjTables<S - 1>::fill(adj);
    }
};
template <>
struct AdjTables<0> {
    static void fill(KernFn (*)[3]) {}
};

template <int S>
struct AdjBatchTables {
    static void fill(void (*(*adj)[2])(const FA*, const int*, int)) {
        adj[S][AM_BETA] = col_adj_batch<S, AM_BETA>;
        adj[S][AM_GAMMA] = col_adj_batch<S, AM_GAMMA>;
        AdjBatchTables<S - 1>::fill(adj);
    }
};
template <>
struct AdjBatchTables<0> {
    static void fill(void (*(*)[2])(const FA*, const int*, int)) {}
};

struct Dispatch {
    KernFn row[MAXS_T + 1];
    KernFn col[MAXS_T + 1][3];
    KernFn adj[MAXS_T + 1][3];
    BatchFn rowb[MAXS_T + 1];
    BatchFn colb[MAXS_T + 1][3];
    BatchFn adjb[MAXS_T + 1][2];
    Dispatch() {
        row[0] = nullptr;
        col[0][0] = col[0][1] = col[0][2] = nullptr;
        adj[0][0] = adj[0][1] = adj[0][2] = nullptr;
        rowb[0] = nullptr;
        colb[0][0] = colb[0][1] = colb[0][2] = nullptr;
        Tables<MAXS_T>::fill(row, col);
        AdjTables<MAXS_T>::fill(adj);
        BatchTables<MAXS_T>::fill(rowb, colb);
        adjb[0][0] = adjb[0][1] = nullptr;
        AdjBatchTables<MAXS_T>::fill(adjb);
    }
};

const Dispatch& dispatch() {
    static Dispatch d;
    return d;
}

// Box windows as running sums (row_box, col_box) or as the unit-tap FIR
// kernels, whichever pass is faster at the radius (measured on 2048 x 2048
// RGB and 1024 x 1024 16-d guides, K 32): the FIR row pass wins below radius
// 26, where its few taps hide behind the coefficient work of the pass, the
// FIR column pass below radius 8.  Beyond the unrolled radii the running
// sums replace the generic tap-by-tap kernels; col_box covers radii up to
// COL_BOX_MAX_S, col_generic the rest.
constexpr int ROW_BOX_MIN_S = 26;
constexpr int COL_BOX_MIN_S = 8;
constexpr int COL_BOX_MAX_S = 64;

bool box_rows(const FilterPlan& fp) { return fp.spatial == FHD_SPATIAL_BOX && fp.S >= ROW_BOX_MIN_S; }
bool box_cols(const FilterPlan& fp) {
    return fp.spatial == FHD_SPATIAL_BOX && fp.S >= COL_BOX_MIN_S && fp.S <= COL_BOX_MAX_S;
}

// Radius tiers of the column running sum (the staged tile has TYC + 2 SB
// rows).

KernFn col_box_kernel(int S, int mode) {
    static const KernFn k[3][3] = {{col_box<16, WM_INLINE>, col_box<16, WM_PLANES>, col_box<16, WM_HARD>},
                                   {col_box<32, WM_INLINE>, col_box<32, WM_PLANES>, col_box<32, WM_HARD>},
                                   {col_box<COL_BOX_MAX_S, WM_INLINE>, col_box<COL_BOX_MAX_S, WM_PLANES>,
                                    col_box<COL_BOX_MAX_S, WM_HARD>}};
    return k[S <= 16 ? 0 : S <= 32 ? 1 : 2][mode];
}

BatchFn col_box_batch_kernel(int S, bool hard) {
    static const BatchFn k[2][2] = {{col_box_batch<16, WM_INLINE>, col_box_batch<16, WM_HARD>},
                                    {col_box_batch<MAXS_T, WM_INLINE>, col_box_batch<MAXS_T, WM_HARD>}};
    return k[S <= 16 ? 0 : 1][hard ? 1 : 0];
}

// The recursive Gaussian of Young and van Vliet (1995), the O(1) Gaussian
// convolution the paper uses (Sec. II-C): q from sigma (two published
// branches, sigma >= 0.5), the polynomial coefficients b0..b3, the gain
// B = 1 - (b1 + b2 + b3) / b0.  c = {B, b1/b0, b2/b0, b3/b0}.
void young_coefficients(double sigma, double* c) {
    const double q = sigma >= 2.5 ? 0.98711 * sigma - 0.96330 : 3.97156 - 4.14554 * std::sqrt(1.0 - 0.26891 * sigma);
    const double q2 = q * q, q3 = q2 * q;
    const double b0 = 1.57825 + 2.44413 * q + 1.4281 * q2 + 0.422205 * q3;
    const double b1 = 2.44413 * q + 2.85619 * q2 + 1.26661 * q3;
    const double b2 = -(1.4281 * q2 + 1.26661 * q3);
    const double b3 = 0.422205 * q3;
    c[0] = 1.0 - (b1 + b2 + b3) / b0;
    c[1] = b1 / b0;
    c[2] = b2 / b0;
    c[3] = b3 / b0;
}

FA make_args(const FilterPlan& fp) {
    FA a;
    std::memset(&a, 0, sizeof(a));
    a.n = fp.n;
    a.rho = fp.rho;
    a.K = fp.K;
    a.H = fp.H;
    a.W = fp.W;
    a.Wp = fp.Wp;
    a.S = fp.S;
    a.coef = fp.coef;
    a.gsplit = 1;
    a.N = fp.N;
    a.Np = (long long)fp.H * fp.Wp;
    a.Pp = (long long)(fp.H + 2 * fp.S) * fp.Wp;
    a.inv2s2 = std::isinf(fp.sigma_r) ? 0.0f : (float)(1.0 / (2.0 * (double)fp.sigma_r * fp.sigma_r));
    if (fp.spatial == FHD_SPATIAL_YOUNG) {
        double yc[4];
        young_coefficients(fp.sigma_s, yc);
        for (int q = 0; q < 4; ++q) a.yc[q] = (float)yc[q];
    }
    for (int j = 0; j <= fp.S; ++j) {
        const bool box = fp.spatial == FHD_SPATIAL_BOX;
        const double s = fp.sigma_s, wj = box ? 1.0 : std::exp(-(double)j * j / (2.0 * s * s));
        a.w[j] = (float)wj;
        a.wd[j] = box ? 0.0f : (float)(wj * j * j / (s * s * s));
    }
    return a;
}

// Intermediate planes: K(n+1) planes of (H + 2S) x Wp, plus slack rows read
// (and discarded) by the last column tile.
size_t plane_floats(const FilterPlan& fp) {
    const size_t Pp = (size_t)(fp.H + 2 * fp.S) * fp.Wp;
    return (size_t)fp.K * (fp.n + 1) * Pp + (size_t)64 * fp.Wp + 64;
}

// Row-pass run length, a multiple of RUN_ALIGN = 32 pixels, so every run
// (and the plane rows it writes, whose pitch Wp is a multiple of 32 floats)
// starts on a 128-byte line.  A run boundary inside a line leaves that line
// written in two parts by two blocks; the row pass's store pattern alone
// measured 0.73 ms for 2.15 GB with 232-pixel runs against 0.48 ms with
// 256-pixel ones.  At radius 8..16 (K <= 32) the runs are 256 pixels and
// the halo run is longer than the block (its first phase takes the rest in
// loops): fewer blocks per row measured 7 % faster at radius 9 and 15.
// Elsewhere the runs are the longest whose halo run fits the 256 threads:
// 256-pixel runs were 5 % slower at radius 1 and 13 % slower at radius 36
// and 60 (the generic kernels).  A row takes the fewest runs of that
// length, of equal length in units of 32 pixels.
constexpr int RUN_ALIGN = 32;

int row_tx(int K, int S, int R, int W) {
    FHD_REQUIRE(RUN_ALIGN % R == 0, FHD_EINVAL, "internal: row task length must divide the run alignment");
    int tx = (K <= 32 && S >= 8 && S <= 16) ? 256 : (RT - 2 * S) / RUN_ALIGN * RUN_ALIGN;
    if (tx < 64) tx = K <= 32 ? 256 : 128;
    const int runs = (W + tx - 1) / tx;
    return std::min(tx, (W + runs * RUN_ALIGN - 1) / (runs * RUN_ALIGN) * RUN_ALIGN);
}

size_t row_lds_bytes(const FilterPlan& fp, int tx) {
    const int hw = tx + 2 * fp.S;
    const int csp = hw + ((hw - 1) >> 3);  // pidx(hw - 1) + 1
    size_t fl = (size_t)fp.K * csp + (size_t)(fp.n + 1) * csp;
    if (!fp.materialize) fl += (size_t)KMAX_INLINE * (RHO_INLINE + KMAX_INLINE);
    return fl * sizeof(float);
}

// The row pass's run length and LDS bytes.  With inline weights every halo
// pixel costs its weights and coefficients, so runs stay long (row_tx); with
// weight planes the halo costs only loads (a few % of the plane writes), so
// runs are shortened until three blocks share a CU's LDS (a 40 KB cap for
// four blocks measured no faster: 44.0 against 44.7 Mpix/s at 512x512x32).
int row_run(const FilterPlan& fp, int R, size_t& lds) {
    int tx = row_tx(fp.K, fp.S, R, fp.W);
    lds = row_lds_bytes(fp, tx);
    const size_t cap = fp.materialize ? 52 * 1024 : 150 * 1024;
    while (lds > cap && tx > RUN_ALIGN) {
        tx -= RUN_ALIGN;
        lds = row_lds_bytes(fp, tx);
    }
    while (lds > 150 * 1024 && tx > RUN_ALIGN) {
        tx -= RUN_ALIGN;
        lds = row_lds_bytes(fp, tx);
    }
    // equal runs again at the shortened length
    const int runs = (fp.W + tx - 1) / tx;
    tx = std::min(tx, (fp.W + runs * RUN_ALIGN - 1) / (runs * RUN_ALIGN) * RUN_ALIGN);
    lds = row_lds_bytes(fp, tx);
    FHD_REQUIRE(lds <= 160 * 1024, FHD_EUNSUPPORTED, "row pass does not fit in LDS");
    return tx;
}

// ---------------------------------------------------------------------------
// 3-D domain (D slices of H x W, flattened to D H rows of the planes): the
// (n+1)K convolutions over the window [-S,S]^3 as three 1-D passes, zero
// outside the volume.  vol_fir_x runs along x, one output position of all
// n + 1 planes of a cluster per thread, forming its input c_l [f, 1] from the
// C planes (or b_l [f, 1] from the B planes, hard variant) on the fly.
// vol_fir_yz runs
// along y within a slice (ax 1) or along z across slices (ax 2, a stride of
// H rows): each thread takes VR consecutive outputs of one column and reads
// the VR + 2S inputs they share once, so a plane element is loaded about
// (VR + 2S) / VR times instead of 2S + 1.  A wave's 64 threads hold adjacent
// x of the same rows (coalesced, and the tap index is wave-uniform).  Taps
// are added in ascending offset order in both.  The planes have no halo
// rows; recomb_young then recombines with b_l.
constexpr int VR = 8;

__global__ __launch_bounds__(RT) void vol_fir_x(FA a, const float* __restrict__ in, float* __restrict__ out) {
    const long long e = (long long)blockIdx.x * RT + threadIdx.x;
    const long long per = (long long)a.H * a.W;  // a.H = D * Hs
    if (e >= (long long)a.K * per) return;
    const int l = (int)(e / per);
    const long long v = e - (long long)l * per;
    const int r = (int)(v / a.W), x = (int)(v - (long long)r * a.W);
    const int S = a.S;
    const float* cb = in + (long long)l * a.Np + (long long)r * a.Wp;
    const int t0 = max(-S, -x), t1 = min(S, a.W - 1 - x);
    // all n + 1 planes of cluster l: the row of c_l is read from the caches
    // after the first channel
    for (int ch = 0; ch <= a.n; ++ch) {
        const float* fb = ch < a.n ? a.f + (long long)ch * a.N + (long long)r * a.W : nullptr;
        float acc = 0.0f;
        for (int t = t0; t <= t1; t += 8) {  // eight taps' loads in flight (addresses clamped into the row)
            float u[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) u[q] = cb[x + min(t + q, t1)];
            if (fb != nullptr) {
                float m[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) m[q] = fb[x + min(t + q, t1)];
#pragma unroll
                for (int q = 0; q < 8; ++q) u[q] *= m[q];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (t + q <= t1) acc = fmaf(a.w[abs(t + q)], u[q], acc);
        }
        out[(long long)(l * (a.n + 1) + ch) * a.Np + (long long)r * a.Wp + x] = acc;
    }
}

__global__ __launch_bounds__(RT) void vol_fir_yz(FA a, int D, int Hs, int ax, const float* __restrict__ in,
                                                float* __restrict__ out) {
    const long long e = (long long)blockIdx.x * RT + threadIdx.x;
    const int planes = a.K * (a.n + 1);
    const int len = ax == 1 ? Hs : D;                    // extent along the axis
    const int ng = (len + VR - 1) / VR;                  // output groups along it
    const int other = ax == 1 ? D : Hs;                  // the remaining row coordinate
    const long long per = (long long)ng * other * a.W;
    if (e >= planes * per) return;
    const int pl = (int)(e / per);
    const long long v = e - (long long)pl * per;
    const int gi = (int)(v / a.W), x = (int)(v - (long long)gi * a.W);
    const int g = gi % ng, o2 = gi / ng;                 // group along the axis, other coordinate
    const int c0 = g * VR;
    // plane row of axis coordinate c
    auto row = [&](int c) { return ax == 1 ? o2 * Hs + c : c * Hs + o2; };
    const float* src = in + (long long)pl * a.Np + x;
    const int S = a.S;
    float acc[VR];
#pragma unroll
    for (int o = 0; o < VR; ++o) acc[o] = 0.0f;
    const int u0 = max(c0 - S, 0), u1 = min(c0 + VR - 1 + S, len - 1);
    for (int u = u0; u <= u1; u += 8) {  // eight inputs' loads in flight (rows clamped into the axis)
        float val[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) val[q] = src[(long long)row(min(u + q, u1)) * a.Wp];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (u + q > u1) break;
#pragma unroll
            for (int o = 0; o < VR; ++o) {
                const int t = u + q - (c0 + o);
                if (t >= -S && t <= S) acc[o] = fmaf(a.w[abs(t)], val[q], acc[o]);
            }
        }
    }
    float* dst = out + (long long)pl * a.Np + x;
#pragma unroll
    for (int o = 0; o < VR; ++o)
        if (c0 + o < len) dst[(long long)row(c0 + o) * a.Wp] = acc[o];
}

// Brute force on a 3-D domain (eqs. (1)-(2) over [-S,S]^3): one thread per
// voxel, the window walked directly (neighbours outside the volume left out),
// omega as the product of the 1-D taps, channels in groups of four (the
// range weights recomputed per group).  FP32, a comparator for the volume
// filter, not on its path.
__global__ __launch_bounds__(RT) void brute_volume(FA a, int D, int Hs, float* __restrict__ out,
                                                  float* __restrict__ den) {
    const long long i = (long long)blockIdx.x * RT + threadIdx.x;
    if (i >= a.N) return;
    const int W = a.W;
    const int x = (int)(i % W);
    const long long zy = i / W;
    const int y = (int)(zy % Hs), z = (int)(zy / Hs);
    const int S = a.S, n = a.n, rho = a.rho;
    const long long N = a.N;
    for (int c0 = 0; c0 < n; c0 += 4) {
        float num[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        float eta = 0.0f;
        for (int jz = -S; jz <= S; ++jz) {
            const int zz = z - jz;
            if (zz < 0 || zz >= D) continue;
            for (int jy = -S; jy <= S; ++jy) {
                const int yy = y - jy;
                if (yy < 0 || yy >= Hs) continue;
                const float wzy = a.w[abs(jz)] * a.w[abs(jy)];
                for (int jx = -S; jx <= S; ++jx) {
                    const int xx = x - jx;
                    if (xx < 0 || xx >= W) continue;
                    const long long q = ((long long)zz * Hs + yy) * W + xx;
                    float d2 = 0.0f;
                    for (int d = 0; d < rho; ++d) {
                        const float t = a.p[d * N + q] - a.p[d * N + i];
                        d2 = fmaf(t, t, d2);
                    }
                    const float w = wzy * a.w[abs(jx)] * __expf(-d2 * a.inv2s2);
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (c0 + k < n) num[k] = fmaf(w, a.f[(c0 + k) * N + q], num[k]);
                    eta += w;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < n) out[(c0 + k) * N + i] = num[k] / eta;
        if (c0 == 0 && den != nullptr) den[i] = eta;
    }
}

// ---------------------------------------------------------------------------
// Error of the kernel approximation at the pixels' own samples: eq. (10)
// evaluated at the method's coefficients c(i) = A^+ b(i),
//   err(i) = sum_{q in window(i), in image} (phi(p(q) - p(i)) - sum_k c_k(i) phi(p(q) - mu_k))^2.
// One thread per pixel (16 x 8 pixels per block).  The centers (zero-padded
// to RM dimensions) and A^+ sit in LDS, and so does each thread's c(i)
// (layout [k][thread]: conflict-free); the pixel's guide vector and each
// neighbour's stay in registers, zero beyond rho (padded dimensions add
// (0 - 0)^2 = 0).  c(i) is formed without storing b(i): each b_k(i) is
// recomputed per row of A^+ (K^2 exponentials against the window's K (2S+1)^2).
// Terms in FP32, sums in FP64; every block writes the FP64 sum of its pixels.
constexpr int AE_X = 16, AE_Y = 8, AE_T = AE_X * AE_Y;

size_t approx_error_lds(int K, int RM) {
    return sizeof(float) * ((size_t)K * RM + (size_t)K * K + (size_t)K * AE_T);
}

template <int RM>
__global__ __launch_bounds__(AE_T) void approx_error_kernel(const float* __restrict__ guide, int rho, int H, int W,
                                                            int K, int S, float inv2s2, const float* __restrict__ mu,
                                                            const float* __restrict__ P, float* __restrict__ err,
                                                            int gx, double* __restrict__ part) {
    extern __shared__ float ae_smem[];
    float* smu = ae_smem;           // K x RM
    float* sP = smu + K * RM;       // K x K
    float* sc = sP + K * K;         // K x AE_T
    __shared__ double red[AE_T / 64];
    const int t = threadIdx.x;
    for (int e = t; e < K * RM; e += AE_T) {
        const int k = e / RM, d = e - k * RM;
        smu[e] = d < rho ? mu[k * rho + d] : 0.0f;
    }
    for (int e = t; e < K * K; e += AE_T) sP[e] = P[e];
    __syncthreads();
    const int bx = (int)(blockIdx.x % gx), by = (int)(blockIdx.x / gx);  // 1-D grid of gx-wide tile rows
    const int x = bx * AE_X + (t % AE_X), y = by * AE_Y + (t / AE_X);
    const long long N = (long long)H * W;
    double acc = 0.0;
    if (x < W && y < H) {
        const long long i = (long long)y * W + x;
        float pi[RM];
#pragma unroll
        for (int d = 0; d < RM; ++d) pi[d] = d < rho ? guide[d * N + i] : 0.0f;
        auto phi_mu = [&](const float (&v)[RM], int k) {
            float s = 0.0f;
#pragma unroll
            for (int d = 0; d < RM; ++d) {
                const float u = v[d] - smu[k * RM + d];
                s = fmaf(u, u, s);
            }
            return __expf(-s * inv2s2);
        };
        for (int l = 0; l < K; ++l) {  // c_l(i) = sum_k A^+_lk b_k(i)
            float s = 0.0f;
            for (int k = 0; k < K; ++k) s = fmaf(sP[l * K + k], phi_mu(pi, k), s);
            sc[l * AE_T + t] = s;
        }
        for (int dy = -S; dy <= S; ++dy) {
            const int yy = y - dy;
            if (yy < 0 || yy >= H) continue;
            for (int dx = -S; dx <= S; ++dx) {
                const int xx = x - dx;
                if (xx < 0 || xx >= W) continue;
                const long long q = (long long)yy * W + xx;
                float xq[RM];
#pragma unroll
                for (int d = 0; d < RM; ++d) xq[d] = d < rho ? guide[d * N + q] : 0.0f;
                float s = 0.0f;
#pragma unroll
                for (int d = 0; d < RM; ++d) {
                    const float u = xq[d] - pi[d];
                    s = fmaf(u, u, s);
                }
                float fit = 0.0f;
                for (int k = 0; k < K; ++k) fit = fmaf(sc[k * AE_T + t], phi_mu(xq, k), fit);
                const double r = (double)(__expf(-s * inv2s2) - fit);
                acc = fma(r, r, acc);
            }
        }
        if (err != nullptr) err[i] = (float)acc;
    }
    double v = acc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        double b = 0.0;
        for (int w = 0; w < AE_T / 64; ++w) b += red[w];
        part[blockIdx.x] = b;
    }
}

}  // namespace

size_t filter_consts_bytes(int K, int rho) {
    return align_up(sizeof(float) * K * rho, 256) + align_up(sizeof(float) * K * K, 256) +
           align_up(sizeof(float) * rho, 256);
}

// centers, A^+ and the contraction offset (mean of the centers), FP32, laid
// out as filter_consts_bytes says, at `dst` (host)
void filter_consts_fill(const float* centers, const float* P32, int K, int rho, char* dst) {
    std::memcpy(dst, centers, sizeof(float) * K * rho);
    std::memcpy(dst + align_up(sizeof(float) * K * rho, 256), P32, sizeof(float) * K * K);
    float* ho = reinterpret_cast<float*>(dst + align_up(sizeof(float) * K * rho, 256) +
                                         align_up(sizeof(float) * K * K, 256));
    for (int d = 0; d < rho; ++d) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += centers[(size_t)k * rho + d];
        ho[d] = (float)(s / K);
    }
}

FilterConsts filter_consts_at(const char* dev, int K, int rho) {
    FilterConsts k;
    k.mu = reinterpret_cast<const float*>(dev);
    k.P = reinterpret_cast<const float*>(dev + align_up(sizeof(float) * K * rho, 256));
    k.offs = reinterpret_cast<const float*>(dev + align_up(sizeof(float) * K * rho, 256) +
                                            align_up(sizeof(float) * K * K, 256));
    return k;
}

size_t filter_passes_workspace(const FilterPlan& fp) {
    Arena probe;
    const long long Np = (long long)fp.H * fp.Wp;
    probe.take<float>(plane_floats(fp));
    if (fp.materialize) {
        probe.take<float>((size_t)fp.K * Np);
        probe.take<float>((size_t)fp.K * Np);
    }
    return probe.used;
}

size_t saved_planes_bytes(const FilterPlan& fp) {
    const size_t kp = align_up(sizeof(float) * (size_t)fp.K * fp.H * fp.Wp, 256);
    return align_up(sizeof(float) * plane_floats(fp), 256) + kp + (fp.materialize ? kp : 0);
}

SavedPlanes saved_at(char* base, const FilterPlan& fp) {
    SavedPlanes s;
    const size_t kp = align_up(sizeof(float) * (size_t)fp.K * fp.H * fp.Wp, 256);
    s.planes = reinterpret_cast<float*>(base);
    s.C = reinterpret_cast<float*>(base + align_up(sizeof(float) * plane_floats(fp), 256));
    s.B = fp.materialize ? reinterpret_cast<float*>(reinterpret_cast<char*>(s.C) + kp) : nullptr;
    return s;
}

size_t filter_workspace(const FilterPlan& fp) {
    return filter_passes_workspace(fp) + filter_consts_bytes(fp.K, fp.rho) + 256;
}

void filter_run(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                const float* centers_host, const float* Pfp32_host, const int* labels, float* out,
                float* den, const SavedPlanes* sv) {
    // stage the constants through pinned memory (async, stream ordered)
    const size_t cb = filter_consts_bytes(fp.K, fp.rho);
    char* dev = ws.take<char>(cb);
    char* hs = static_cast<char*>(c.host_stage(1, cb));
    filter_consts_fill(centers_host, Pfp32_host, fp.K, fp.rho, hs);
    FHD_HIP(hipMemcpyAsync(dev, hs, cb, hipMemcpyHostToDevice, c.stream));
    c.stage_done(1);
    filter_passes(c, ws, fp, f, guide, filter_consts_at(dev, fp.K, fp.rho), labels, out, den, sv);
}

void filter_passes(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                   const FilterConsts& kc, const int* labels, float* out, float* den, const SavedPlanes* sv) {
    const long long Np = (long long)fp.H * fp.Wp;
    FHD_REQUIRE(sv == nullptr || (fp.S >= 1 && fp.S <= MAXS_T && fp.spatial != FHD_SPATIAL_YOUNG &&
                                  fp.coef == FHD_COEF_LSQ && fp.contract == FHD_CONTRACT_FP32),
                FHD_EINVAL, "internal: saved planes need the adjoint's window, FP32 and least squares");
    float* planes = sv != nullptr ? sv->planes : ws.take<float>(plane_floats(fp));
    float* Bpl = nullptr;
    float* Cpl = nullptr;
    if (fp.materialize) {
        Bpl = sv != nullptr ? sv->B : ws.take<float>((size_t)fp.K * Np);
        Cpl = sv != nullptr ? sv->C : ws.take<float>((size_t)fp.K * Np);
    }
    const float* mu = kc.mu;
    const float* P = kc.P;
    const float* offs = kc.offs;
    hipStream_t st = c.stream;

    FA a = make_args(fp);
    a.f = f;
    a.p = guide;
    a.mu = mu;
    a.P = P;
    a.labels = labels;
    a.planes = planes;
    a.out = out;
    a.den = den;
    a.Csave = (sv != nullptr && !fp.materialize) ? sv->C : nullptr;

    if (fp.materialize && fp.contract != FHD_CONTRACT_FP32) {
        const size_t plds = sizeof(float) * (size_t)fp.K * pad8(fp.K);
        const void* wk = fp.contract == FHD_CONTRACT_BF16 ? reinterpret_cast<const void*>(weights_mfma<true>)
                                                          : reinterpret_cast<const void*>(weights_mfma<false>);
        FHD_HIP(hipFuncSetAttribute(wk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds));
        hipEvent_t tw = c.stage_begin();
        const dim3 g((fp.W + MW_PIX - 1) / MW_PIX, fp.H);
        if (fp.contract == FHD_CONTRACT_BF16)
            hipLaunchKernelGGL(weights_mfma<true>, g, dim3(RT), plds, st, a, Bpl,
                               fp.coef == FHD_COEF_HARD ? nullptr : Cpl, offs);
        else
            hipLaunchKernelGGL(weights_mfma<false>, g, dim3(RT), plds, st, a, Bpl,
                               fp.coef == FHD_COEF_HARD ? nullptr : Cpl, offs);
        FHD_HIP(hipGetLastError());
        c.stage_end(FHD_STAGE_WEIGHTS, tw);
        a.Bpl = Bpl;
        a.Cpl = Cpl;
    } else if (fp.materialize) {
        const int npx = weights_fp32_npx(fp.K);
        const size_t lds = weights_fp32_lds(fp.K, fp.rho, npx);
        FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(weights_fp32),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipEvent_t tw = c.stage_begin();
        hipLaunchKernelGGL(weights_fp32, dim3((fp.W + npx - 1) / npx, fp.H), dim3(npx), lds, st, a, Bpl,
                           fp.coef == FHD_COEF_HARD ? nullptr : Cpl);
        c.stage_end(FHD_STAGE_WEIGHTS, tw);
        FHD_HIP(hipGetLastError());
        a.Bpl = Bpl;
        a.Cpl = Cpl;
        if (fp.coef == FHD_COEF_EXACT) {
            // the per-pixel fit of eq. (10) replaces c = A^+ b.  The passes
            // convolve c_l [f, 1] and recombine with b_l(i), which equals
            // eqs. (13)-(16) only for c = A^+ b with A^+ symmetric; here they
            // run as written: the row pass convolves b_k [f, 1] (the B planes
            // as its factor) and the column pass recombines with c*_k(i)
            // (the C planes as its weights).
            exact_ls_run(c, guide, fp.rho, fp.H, fp.W, mu, fp.K, nullptr, fp.sigma_r, fp.S, Cpl, Np, fp.Wp, nullptr,
                         nullptr);
            a.Bpl = Cpl;
            a.Cpl = Bpl;
        }
    }

    if (fp.spatial == FHD_SPATIAL_YOUNG) {  // recursive Gaussian (materialised weights, S = 0)
        const bool hard = fp.coef == FHD_COEF_HARD;
        const long long planes = (long long)fp.K * (fp.n + 1);
        const long long nr = planes * ((fp.H + YT - 1) / YT), nc = planes * fp.W;
        FHD_REQUIRE(nr < (1LL << 31) && (nc + RT - 1) / RT < (1LL << 31), FHD_EUNSUPPORTED,
                    "too many plane rows for the recursive passes");
        hipEvent_t ty = c.stage_begin();
        hipLaunchKernelGGL(row_young, dim3((unsigned)nr), dim3(YT), 0, st, a, hard ? Bpl : Cpl);
        c.stage_end(FHD_STAGE_ROW, ty);
        ty = c.stage_begin();
        hipLaunchKernelGGL(col_young, dim3((unsigned)((nc + RT - 1) / RT)), dim3(RT), 0, st, a);
        hipLaunchKernelGGL(recomb_young, dim3((unsigned)((fp.N + RT - 1) / RT)), dim3(RT), 0, st, a, hard ? 1 : 0);
        c.stage_end(FHD_STAGE_COL, ty);
        FHD_HIP(hipGetLastError());
        return;
    }

    // (the S zero rows above and below every plane come from the row pass)
    // row pass
    const bool box = fp.spatial == FHD_SPATIAL_BOX;
    // radii 1..32 take the unrolled register-window kernels (a box is the
    // window with every tap 1); the generic kernels cover the rest
    const bool unrolled = fp.S >= 1 && fp.S <= MAXS_T;
    const int rR = unrolled ? R_ROW : 16;
    size_t lds = 0;
    const int tx = row_run(fp, rR, lds);
    a.tx = tx;
    FHD_REQUIRE(fp.H + 2 * fp.S <= 65535, FHD_EUNSUPPORTED, "image height plus 2 radius exceeds 65535");
    const dim3 rg((fp.W + tx - 1) / tx, fp.H + 2 * fp.S);
    KernFn rowk = box_rows(fp) ? row_box
                  : unrolled   ? dispatch().row[fp.S]
                               : (box ? row_generic<true> : row_generic<false>);
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(rowk),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipEvent_t tr = c.stage_begin();
    hipLaunchKernelGGL(rowk, rg, dim3(RT), lds, st, a);
    c.stage_end(FHD_STAGE_ROW, tr);
    FHD_HIP(hipGetLastError());

    // column pass + recombination
    // the double-buffered tile kernels (col_body): unrolled radii, and box
    // windows up to COL_BOX_MAX_S as running sums
    const bool colbox = box_cols(fp);
    const bool tiled = unrolled || colbox;
    const int ty = tiled ? TYC : 16 * (RT / TXC);
    const int gx = (fp.W + TXC - 1) / TXC, gy = (fp.H + ty - 1) / ty;
    const int total = gx * gy;
    const int per = (total + 7) / 8;
    a.xcd_groups = per;
    // too few tiles to fill the chip: split each tile's channel groups over
    // several blocks (each extra part also filters the normaliser planes)
    const int groups = (fp.n + 1 + CG - 1) / CG;
    a.gsplit = tiled ? std::max(1, std::min(groups, 1024 / (per * 8))) : 1;
    const dim3 cg(per * 8 * a.gsplit);
    size_t clds = (fp.materialize || fp.coef == FHD_COEF_HARD) ? 0 : sizeof(float) * fp.rho * ty * TXC;
    if (!tiled) clds += sizeof(float) * (size_t)(ty + 2 * fp.S) * TXC;
    const int mode = fp.coef == FHD_COEF_HARD ? WM_HARD : (fp.materialize ? WM_PLANES : WM_INLINE);
    static const KernFn gen[2][3] = {
        {col_generic<false, WM_INLINE>, col_generic<false, WM_PLANES>, col_generic<false, WM_HARD>},
        {col_generic<true, WM_INLINE>, col_generic<true, WM_PLANES>, col_generic<true, WM_HARD>}};
    KernFn colk = colbox ? col_box_kernel(fp.S, mode) : unrolled ? dispatch().col[fp.S][mode] : gen[box ? 1 : 0][mode];
    FHD_REQUIRE(clds <= 150 * 1024, FHD_EUNSUPPORTED, "column pass does not fit in LDS");
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(colk),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)clds));
    hipEvent_t tc = c.stage_begin();
    hipLaunchKernelGGL(colk, cg, dim3(RT), clds, st, a);
    c.stage_end(FHD_STAGE_COL, tc);
    FHD_HIP(hipGetLastError());
}

bool filter_batch_supported(const FilterPlan& fp) {
    return !fp.materialize && fp.S >= 1 && fp.S <= MAXS_T;
}

size_t filter_batch_workspace(int B, const FilterPlan* plans) {
    Arena probe;
    for (int b = 0; b < B; ++b) probe.take<float>(plane_floats(plans[b]));
    probe.take<FA>((size_t)B);
    probe.take<int>(2 * (size_t)(B + 1));
    return probe.used;
}

// The row and column passes of every image of a batch, one launch each for
// all images (images of at most 8 guide dimensions and 32 clusters, radius
// 1..32: weights inline).
void filter_passes_batch(Ctx& c, Arena& ws, int B, const FilterPlan* plans, const float* const* f,
                         const float* const* guide, const FilterConsts* kc, const int* const* labels,
                         float* const* out, float* const* den, const SavedPlanes* sv) {
    const int S = plans[0].S;
    const bool hard = plans[0].coef == FHD_COEF_HARD;
    std::vector<FA> fas(B);
    std::vector<int> pre_row(B + 1, 0), pre_col(B + 1, 0);
    size_t lds = 0;
    for (int b = 0; b < B; ++b) {
        const FilterPlan& fp = plans[b];
        FHD_REQUIRE(filter_batch_supported(fp) && fp.S == S && (fp.coef == FHD_COEF_HARD) == hard &&
                        fp.spatial == plans[0].spatial,
                    FHD_EINVAL, "internal: batch plans differ");
        FHD_REQUIRE(fp.H + 2 * fp.S <= 65535, FHD_EUNSUPPORTED, "image height plus 2 radius exceeds 65535");
        FA& a = fas[b];
        a = make_args(fp);
        a.f = f[b];
        a.p = guide[b];
        a.mu = kc[b].mu;
        a.P = kc[b].P;
        a.labels = labels ? labels[b] : nullptr;
        a.planes = sv != nullptr ? sv[b].planes : ws.take<float>(plane_floats(fp));
        a.Csave = sv != nullptr ? sv[b].C : nullptr;
        a.out = out[b];
        a.den = den ? den[b] : nullptr;
        size_t l = 0;
        const int tx = row_run(fp, R_ROW, l);
        lds = std::max(lds, l);
        a.tx = tx;
        pre_row[b + 1] = pre_row[b] + ((fp.W + tx - 1) / tx) * (fp.H + 2 * fp.S);
        const int gx = (fp.W + TXC - 1) / TXC, gy = (fp.H + TYC - 1) / TYC;
        a.xcd_groups = (gx * gy + 7) / 8;
        a.gsplit = 1;
        pre_col[b + 1] = pre_col[b] + a.xcd_groups * 8;
    }
    FA* dfa = ws.take<FA>((size_t)B);
    int* dpre = ws.take<int>(2 * (size_t)(B + 1));
    const size_t fab = sizeof(FA) * B, prb = sizeof(int) * (B + 1);
    char* hs = static_cast<char*>(c.host_stage(2, align_up(fab, 256) + 2 * prb));
    std::memcpy(hs, fas.data(), fab);
    std::memcpy(hs + align_up(fab, 256), pre_row.data(), prb);
    std::memcpy(hs + align_up(fab, 256) + prb, pre_col.data(), prb);
    hipStream_t st = c.stream;
    FHD_HIP(hipMemcpyAsync(dfa, hs, fab, hipMemcpyHostToDevice, st));
    FHD_HIP(hipMemcpyAsync(dpre, hs + align_up(fab, 256), 2 * prb, hipMemcpyHostToDevice, st));
    c.stage_done(2);
    BatchFn rowk = box_rows(plans[0]) ? row_box_batch : dispatch().rowb[S];
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(rowk), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipEvent_t t0 = c.stage_begin();
    hipLaunchKernelGGL(rowk, dim3(pre_row[B]), dim3(RT), lds, st, (const FA*)dfa, (const int*)dpre, B);
    c.stage_end(FHD_STAGE_ROW, t0);
    FHD_HIP(hipGetLastError());
    const int mode = hard ? WM_HARD : WM_INLINE;
    const size_t clds = hard ? 0 : sizeof(float) * plans[0].rho * TYC * TXC;
    BatchFn colk = box_cols(plans[0]) ? col_box_batch_kernel(S, hard) : dispatch().colb[S][mode];
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(colk), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)clds));
    t0 = c.stage_begin();
    hipLaunchKernelGGL(colk, dim3(pre_col[B]), dim3(RT), clds, st, (const FA*)dfa, (const int*)(dpre + B + 1), B);
    c.stage_end(FHD_STAGE_COL, t0);
    FHD_HIP(hipGetLastError());
}

size_t adjoint_consts_bytes(int K, int rho) {
    return filter_consts_bytes(K, rho) + align_up(sizeof(float) * K * K, 256);
}

int centers_sum_entries(int K, int rho) { return K * K + K + K * rho; }

size_t adjoint_passes_workspace(const FilterPlan& fp, bool with_s, bool with_mu) {
    Arena probe;
    const long long Np = (long long)fp.H * fp.Wp;
    probe.take<float>(plane_floats(fp));
    for (int q = 0; q < (with_s ? 5 : 4); ++q) probe.take<float>((size_t)fp.K * Np);
    probe.take<double>(2 * ((size_t)(fp.N + RT - 1) / RT) + 1);
    if (with_s) probe.take<double>(2 * ((size_t)(fp.N + RT - 1) / RT) + 1);
    if (with_mu) probe.take<double>((size_t)MU_GRID * centers_sum_entries(fp.K, fp.rho));
    return probe.used;
}

size_t adjoint_workspace(const FilterPlan& fp, bool with_s, bool with_mu) {
    return adjoint_passes_workspace(fp, with_s, with_mu) + adjoint_consts_bytes(fp.K, fp.rho) +
           align_up(sizeof(double) * (2 + (size_t)centers_sum_entries(fp.K, fp.rho)), 256) + 512;
}

// adj_final_mfma addresses a K-plane set and the guide with 32-bit byte offsets
bool adj_final_mfma_fits(const FilterPlan& fp) {
    const long long Np = (long long)fp.H * fp.Wp;
    return (long long)fp.K * Np * 4 < (1LL << 32) && fp.N * fp.rho * 4 < (1LL << 32);
}

void adjoint_run(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                 const float* centers_host, const float* Pfp32_host, const float* M_host, const float* out,
                 const float* den, const float* gout, float* gradf, float* gradp, double* gsig, double* gsigs,
                 double rtol, double* gmu, const SavedPlanes* sv) {
    const size_t cb = adjoint_consts_bytes(fp.K, fp.rho);
    char* dev = ws.take<char>(cb);
    char* hs = static_cast<char*>(c.host_stage(1, cb));
    filter_consts_fill(centers_host, Pfp32_host, fp.K, fp.rho, hs);
    std::memcpy(hs + filter_consts_bytes(fp.K, fp.rho), M_host, sizeof(float) * fp.K * fp.K);
    FHD_HIP(hipMemcpyAsync(dev, hs, cb, hipMemcpyHostToDevice, c.stream));
    c.stage_done(1);
    const int E = centers_sum_entries(fp.K, fp.rho);
    double* sig = ws.take<double>(2 + (size_t)E);
    adjoint_passes(c, ws, fp, f, guide, filter_consts_at(dev, fp.K, fp.rho),
                   reinterpret_cast<const float*>(dev + filter_consts_bytes(fp.K, fp.rho)), out, den, gout, gradf,
                   gradp, sig, gsigs != nullptr ? sig + 1 : nullptr, gmu != nullptr ? sig + 2 : nullptr, sv);
    if (gsig != nullptr || gsigs != nullptr || gmu != nullptr) {
        std::vector<double> h(2 + (size_t)E);
        FHD_HIP(hipMemcpyAsync(h.data(), sig, sizeof(double) * (gmu != nullptr ? 2 + E : 2), hipMemcpyDeviceToHost,
                               c.stream));
        FHD_HIP(hipStreamSynchronize(c.stream));
        if (gsig != nullptr) *gsig = h[0];
        if (gsigs != nullptr) *gsigs = h[1];
        if (gmu != nullptr) {
            const int K = fp.K, rho = fp.rho;
            const double* Gm = h.data() + 2;
            centers_gradient(centers_host, K, rho, fp.sigma_r, rtol, Gm, Gm + (size_t)K * K,
                             Gm + (size_t)K * K + K, gmu);
        }
    }
}

void adjoint_passes(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                    const FilterConsts& kc, const float* Md, const float* out, const float* den, const float* gout,
                    float* gradf, float* gradp, double* sig_dev, double* sigs_dev, double* mu_dev,
                    const SavedPlanes* sv) {
    FHD_REQUIRE(fp.S >= 1 && fp.S <= MAXS_T, FHD_EUNSUPPORTED, "the adjoint supports radii 1..32");
    FHD_REQUIRE(fp.K <= 64, FHD_EUNSUPPORTED, "the adjoint supports K <= 64");
    FHD_REQUIRE(fp.coef == FHD_COEF_LSQ, FHD_EUNSUPPORTED, "the adjoint covers least-squares coefficients");
    FHD_REQUIRE(fp.materialize, FHD_EINVAL, "internal: adjoint plan must materialise weights");
    const long long Np = (long long)fp.H * fp.Wp;
    float* planes = ws.take<float>(plane_floats(fp));
    // with the forward's saved intermediates: its row-filtered planes of
    // c_l [f, 1] (the first row pass below) and its C (and B) planes (the
    // weights pass) are reused
    float* Bpl = ws.take<float>((size_t)fp.K * Np);
    float* Cpl = ws.take<float>((size_t)fp.K * Np);
    if (sv != nullptr) {
        Cpl = sv->C;
        if (sv->B != nullptr) Bpl = sv->B;
    }
    float* beta = ws.take<float>((size_t)fp.K * Np);
    float* gamma = ws.take<float>((size_t)fp.K * Np);
    const int nb = (int)((fp.N + RT - 1) / RT);
    double* part = ws.take<double>(2 * (size_t)nb + 1);
    const bool with_s = sigs_dev != nullptr;
    FHD_REQUIRE(!with_s || fp.spatial == FHD_SPATIAL_GAUSSIAN, FHD_EUNSUPPORTED,
                "dL/dsigma_s needs the Gaussian spatial kernel");
    float* betas = with_s ? ws.take<float>((size_t)fp.K * Np) : nullptr;
    double* parts = with_s ? ws.take<double>(2 * (size_t)nb + 1) : nullptr;
    const int Emu = centers_sum_entries(fp.K, fp.rho);
    const size_t mulds = adj_centers_lds(fp.K, fp.rho);
    FHD_REQUIRE(mu_dev == nullptr || mulds <= 160 * 1024, FHD_EUNSUPPORTED,
                "dL/dcenters: K x K plus K x rho sums do not fit in LDS");
    double* mupart = mu_dev != nullptr ? ws.take<double>((size_t)MU_GRID * Emu) : nullptr;
    hipStream_t st = c.stream;

    FA a = make_args(fp);
    a.f = f;
    a.p = guide;
    a.mu = kc.mu;
    a.P = kc.P;
    a.planes = planes;
    a.gout = gout;
    a.gimg = out;
    a.gden = den;
    a.beta = beta;
    a.gamma = gamma;
    a.gradf = gradf;
    // Weights recomputed from the guide (never stored by the forward call).
    // Short guides (the inline case of the forward pass) keep only the C
    // planes: the row passes form c and b per halo pixel as the forward row
    // pass does, and the final kernel recomputes b.
    const bool inl = fp.rho <= RHO_INLINE && fp.K <= KMAX_INLINE;
    FHD_REQUIRE(sv == nullptr || inl == (sv->B == nullptr), FHD_EINVAL,
                "internal: saved planes were written for the other weights layout");
    if (sv == nullptr) {
        const int npx = weights_fp32_npx(fp.K);
        const size_t lds = weights_fp32_lds(fp.K, fp.rho, npx);
        FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(weights_fp32),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipEvent_t tw = c.stage_begin();
        hipLaunchKernelGGL(weights_fp32, dim3((fp.W + npx - 1) / npx, fp.H), dim3(npx), lds, st, a,
                           inl ? nullptr : Bpl, Cpl);
        c.stage_end(FHD_STAGE_WEIGHTS, tw);
        FHD_HIP(hipGetLastError());
    }
    a.Bpl = inl ? nullptr : Bpl;
    a.Cpl = inl ? nullptr : Cpl;   // row passes: null = factors formed inline
    FilterPlan rp = fp;
    rp.materialize = !inl;
    size_t lds = 0;
    const int tx = row_run(rp, R_ROW, lds);
    a.tx = tx;
    FHD_REQUIRE(fp.H + 2 * fp.S <= 65535, FHD_EUNSUPPORTED, "image height plus 2 radius exceeds 65535");
    const dim3 rg((fp.W + tx - 1) / tx, fp.H + 2 * fp.S);
    KernFn rowk = box_rows(fp) ? row_box : dispatch().row[fp.S];  // the forward's row kernel
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(rowk), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    const int gx = (fp.W + TXC - 1) / TXC, gy = (fp.H + TYC - 1) / TYC;
    const int per = (gx * gy + 7) / 8;
    a.xcd_groups = per;
    const dim3 cg(per * 8);
    // dL/db_l from the recombination: Q_l = w * (c_l [f, 1]), its row half
    // saved by the forward call or recomputed here
    a.fmode = 0;
    a.factor_b = 0;
    hipEvent_t t0 = nullptr;
    if (sv != nullptr) {
        a.planes = sv->planes;
    } else {
        t0 = c.stage_begin();
        hipLaunchKernelGGL(rowk, rg, dim3(RT), lds, st, a);
        c.stage_end(FHD_STAGE_ROW, t0);
    }
    t0 = c.stage_begin();
    if (with_s) {
        // beta_l, and the first half of (d omega / d sigma_s) = w' (x) w + w (x) w':
        // the column derivative taps on the same row-filtered planes
        a.betas = betas;
        hipLaunchKernelGGL(dispatch().adj[fp.S][AM_BETAS], cg, dim3(RT), 0, st, a);
        c.stage_end(FHD_STAGE_COL, t0);
        // the second half: row derivative taps, then the column taps, added
        FA ad = a;
        ad.planes = planes;
        for (int j = 0; j <= fp.S; ++j) ad.w[j] = a.wd[j];
        t0 = c.stage_begin();
        hipLaunchKernelGGL(rowk, rg, dim3(RT), lds, st, ad);
        c.stage_end(FHD_STAGE_ROW, t0);
        FA ab = a;
        ab.planes = planes;
        ab.beta = betas;
        ab.betas = nullptr;
        ab.bacc = 1;
        t0 = c.stage_begin();
        hipLaunchKernelGGL(dispatch().adj[fp.S][AM_BETA], cg, dim3(RT), 0, st, ab);
    } else {
        hipLaunchKernelGGL(dispatch().adj[fp.S][AM_BETA], cg, dim3(RT), 0, st, a);
    }
    c.stage_end(FHD_STAGE_COL, t0);
    // the adjoint convolution of dL/dQ_l = b_l Y
    a.planes = planes;
    a.fmode = 1;
    a.factor_b = 1;
    t0 = c.stage_begin();
    hipLaunchKernelGGL(rowk, rg, dim3(RT), lds, st, a);
    c.stage_end(FHD_STAGE_ROW, t0);
    a.Cpl = Cpl;  // the GAMMA epilogue multiplies by c_l(i)
    t0 = c.stage_begin();
    hipLaunchKernelGGL(dispatch().adj[fp.S][AM_GAMMA], cg, dim3(RT), 0, st, a);
    c.stage_end(FHD_STAGE_COL, t0);
    FHD_HIP(hipGetLastError());
    const float sig3inv =
        std::isinf(fp.sigma_r) ? 0.0f : (float)(1.0 / ((double)fp.sigma_r * fp.sigma_r * fp.sigma_r));
    if (inl && adj_final_mfma_fits(fp)) {  // rho <= 8, K <= 32: the matrix-core form
        const int nb32 = (int)((fp.N + AF_PIX - 1) / AF_PIX);
        hipLaunchKernelGGL(adj_final_mfma, dim3(nb32), dim3(RT), 0, st, a, Md, sig3inv, gradp, part,
                           with_s ? parts : nullptr);
        hipLaunchKernelGGL(sum_blocks, dim3(1), dim3(RT), 0, st, part, nb32, sig_dev);
        if (with_s) hipLaunchKernelGGL(sum_blocks, dim3(1), dim3(RT), 0, st, parts, nb32, sigs_dev);
    } else {
        const int halves = (fp.K + KF - 1) / KF;
        for (int h = 0; h < halves; ++h)
            hipLaunchKernelGGL(adj_final, dim3(nb), dim3(RT), 0, st, a, Md, sig3inv, h * KF, h, gradp,
                               part + (size_t)h * nb, with_s ? parts + (size_t)h * nb : nullptr);
        hipLaunchKernelGGL(sum_blocks, dim3(1), dim3(RT), 0, st, part, halves * nb, sig_dev);
        if (with_s) hipLaunchKernelGGL(sum_blocks, dim3(1), dim3(RT), 0, st, parts, halves * nb, sigs_dev);
    }
    if (mu_dev != nullptr) {
        // the pixel sums of the centers gradient (beta and gamma are complete)
        FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(adj_centers),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mulds));
        hipLaunchKernelGGL(adj_centers, dim3(MU_GRID), dim3(CMU), mulds, st, a, mupart);
        hipLaunchKernelGGL(sum_entries, dim3((Emu + RT - 1) / RT), dim3(RT), 0, st, mupart, MU_GRID, Emu, mu_dev);
    }
    FHD_HIP(hipGetLastError());
}

bool adjoint_batch_supported(const FilterPlan& fp) {
    return fp.S >= 1 && fp.S <= MAXS_T && fp.rho <= RHO_INLINE && fp.K <= KMAX_INLINE &&
           fp.coef == FHD_COEF_LSQ && fp.H + 2 * fp.S <= 65535 && adj_final_mfma_fits(fp);
}

size_t adjoint_batch_workspace(int B, const FilterPlan* plans) {
    Arena probe;
    long long nb = 0;
    for (int b = 0; b < B; ++b) {
        const long long Np = (long long)plans[b].H * plans[b].Wp;
        probe.take<float>(plane_floats(plans[b]));
        for (int q = 0; q < 3; ++q) probe.take<float>((size_t)plans[b].K * Np);
        nb += (plans[b].N + RT - 1) / RT;
    }
    probe.take<double>((size_t)nb + 1);
    probe.take<FA>(3 * (size_t)B);
    probe.take<int>(4 * (size_t)(B + 1));
    return probe.used;
}

// The adjoint of every image of a batch with one launch per pass for all
// images (guides of at most 8 dimensions, at most 32 clusters, radius 1..32:
// the weights b are formed inline, only the C planes are stored).  Three
// tables of per-image arguments: the first row pass (c_l [f, 1]), the second
// row pass (b_l Y), and the weights / GAMMA / final passes, which read the
// C planes.  The block partials of dL/dsigma_r of all images are summed into
// sig_dev.
void adjoint_passes_batch(Ctx& c, Arena& ws, int B, const FilterPlan* plans, const float* const* f,
                          const float* const* guide, const FilterConsts* kc, const float* const* Md,
                          const float* const* out, const float* const* den, const float* const* gout,
                          float* const* gradf, float* const* gradp, double* sig_dev, const SavedPlanes* sv) {
    const int S = plans[0].S;
    std::vector<FA> fas(3 * (size_t)B);
    std::vector<int> pre(4 * (size_t)(B + 1), 0);
    int* pre_w = pre.data();
    int* pre_r = pre_w + (B + 1);
    int* pre_c = pre_r + (B + 1);
    int* pre_f = pre_c + (B + 1);
    size_t rlds = 0, wlds = 0;
    const int npx = RT;
    for (int b = 0; b < B; ++b) {
        const FilterPlan& fp = plans[b];
        FHD_REQUIRE(adjoint_batch_supported(fp) && fp.S == S && fp.sigma_r == plans[0].sigma_r &&
                        fp.spatial == plans[0].spatial,
                    FHD_EINVAL, "internal: batch adjoint plans differ");
        FHD_REQUIRE(weights_fp32_npx(fp.K) == npx, FHD_EINVAL, "internal: weights block size");
        const long long Np = (long long)fp.H * fp.Wp;
        FA a = make_args(fp);
        a.f = f[b];
        a.p = guide[b];
        a.mu = kc[b].mu;
        a.P = kc[b].P;
        a.planes = ws.take<float>(plane_floats(fp));
        float* Cpl = ws.take<float>((size_t)fp.K * Np);
        if (sv != nullptr) Cpl = sv[b].C;
        a.beta = ws.take<float>((size_t)fp.K * Np);
        a.gamma = ws.take<float>((size_t)fp.K * Np);
        a.gout = gout[b];
        a.gimg = out[b];
        a.gden = den[b];
        a.gradf = gradf[b];
        a.Md = Md[b];
        a.gradp = gradp[b];
        a.Bpl = nullptr;
        a.Cpl = nullptr;
        FilterPlan rp = fp;
        rp.materialize = false;
        size_t l = 0;
        const int tx = row_run(rp, R_ROW, l);
        rlds = std::max(rlds, l);
        wlds = std::max(wlds, weights_fp32_lds(fp.K, fp.rho, npx));
        a.tx = tx;
        const int gx = (fp.W + TXC - 1) / TXC, gy = (fp.H + TYC - 1) / TYC;
        a.xcd_groups = (gx * gy + 7) / 8;
        a.gsplit = 1;
        a.fmode = 0;
        a.factor_b = 0;
        fas[b] = a;                 // first row pass, BETA column pass
        if (sv != nullptr) fas[b].planes = sv[b].planes;  // the forward's row-filtered planes
        a.fmode = 1;
        a.factor_b = 1;
        fas[B + b] = a;             // second row pass
        a.Cpl = Cpl;
        fas[2 * (size_t)B + b] = a; // weights (C planes), GAMMA column pass, final pass
        pre_w[b + 1] = pre_w[b] + ((fp.W + npx - 1) / npx) * fp.H;
        pre_r[b + 1] = pre_r[b] + ((fp.W + tx - 1) / tx) * (fp.H + 2 * fp.S);
        pre_c[b + 1] = pre_c[b] + a.xcd_groups * 8;
        pre_f[b + 1] = pre_f[b] + (int)((fp.N + AF_PIX - 1) / AF_PIX);
    }
    double* part = ws.take<double>((size_t)pre_f[B] + 1);
    FA* dfa = ws.take<FA>(3 * (size_t)B);
    int* dpre = ws.take<int>(4 * (size_t)(B + 1));
    const size_t fab = sizeof(FA) * 3 * B, prb = sizeof(int) * 4 * (B + 1);
    char* hs = static_cast<char*>(c.host_stage(2, align_up(fab, 256) + prb));
    std::memcpy(hs, fas.data(), fab);
    std::memcpy(hs + align_up(fab, 256), pre.data(), prb);
    hipStream_t st = c.stream;
    FHD_HIP(hipMemcpyAsync(dfa, hs, fab, hipMemcpyHostToDevice, st));
    FHD_HIP(hipMemcpyAsync(dpre, hs + align_up(fab, 256), prb, hipMemcpyHostToDevice, st));
    c.stage_done(2);
    const FA* fa0 = dfa;
    const FA* fa1 = dfa + B;
    const FA* fa2 = dfa + 2 * B;
    const int* dw = dpre;
    const int* dr = dpre + (B + 1);
    const int* dc = dpre + 2 * (B + 1);
    const int* df = dpre + 3 * (B + 1);
    hipEvent_t t0 = nullptr;
    if (sv == nullptr) {  // else the forward's C planes
        FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(weights_fp32_batch),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)wlds));
        t0 = c.stage_begin();
        hipLaunchKernelGGL(weights_fp32_batch, dim3(pre_w[B]), dim3(npx), wlds, st, fa2, dw, B);
        c.stage_end(FHD_STAGE_WEIGHTS, t0);
        FHD_HIP(hipGetLastError());
    }
    BatchFn rowk = box_rows(plans[0]) ? row_box_batch : dispatch().rowb[S];  // the forward's row kernel
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(rowk), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)rlds));
    // dL/db_l from the recombination: Q_l = w * (c_l [f, 1]), its row half
    // saved by the forward call or recomputed here
    if (sv == nullptr) {
        t0 = c.stage_begin();
        hipLaunchKernelGGL(rowk, dim3(pre_r[B]), dim3(RT), rlds, st, fa0, dr, B);
        c.stage_end(FHD_STAGE_ROW, t0);
    }
    t0 = c.stage_begin();
    hipLaunchKernelGGL(dispatch().adjb[S][AM_BETA], dim3(pre_c[B]), dim3(RT), 0, st, fa0, dc, B);
    c.stage_end(FHD_STAGE_COL, t0);
    // the adjoint convolution of dL/dQ_l = b_l Y
    t0 = c.stage_begin();
    hipLaunchKernelGGL(rowk, dim3(pre_r[B]), dim3(RT), rlds, st, fa1, dr, B);
    c.stage_end(FHD_STAGE_ROW, t0);
    t0 = c.stage_begin();
    hipLaunchKernelGGL(dispatch().adjb[S][AM_GAMMA], dim3(pre_c[B]), dim3(RT), 0, st, fa2, dc, B);
    c.stage_end(FHD_STAGE_COL, t0);
    FHD_HIP(hipGetLastError());
    const float sig3inv = std::isinf(plans[0].sigma_r)
                              ? 0.0f
                              : (float)(1.0 / ((double)plans[0].sigma_r * plans[0].sigma_r * plans[0].sigma_r));
    hipLaunchKernelGGL(adj_final_mfma_batch, dim3(pre_f[B]), dim3(RT), 0, st, fa2, df, B, sig3inv, part);
    hipLaunchKernelGGL(sum_blocks, dim3(1), dim3(RT), 0, st, part, pre_f[B], sig_dev);
    FHD_HIP(hipGetLastError());
}

void sum_doubles(Ctx& c, const double* v, int count, double* out_dev) {
    hipLaunchKernelGGL(sum_blocks, dim3(1), dim3(RT), 0, c.stream, v, count, out_dev);
    FHD_HIP(hipGetLastError());
}

void bruteforce_run(Ctx& c, const FilterPlan& fp, const float* f, const float* guide, float* out,
                    float* den) {
    FA a = make_args(fp);
    a.f = f;
    a.p = guide;
    a.out = out;
    a.den = den;
    // the variant for the channel counts, rows per thread R as measured (RGB:
    // R 8 3.39 ms at 2048x2048, S 15, R 16 5.06 ms at 150 VGPRs; 16-d guide
    // and RGB image: R 8 1.19 ms at 1024x1024, S 10, R 4 1.75 ms)
    const bool same = f == guide && fp.n == fp.rho;
    KernFn k;
    int R;
    if (fp.rho == 3 && fp.n == 3) {
        k = same ? brute_strip<8, 3, 3, true, true> : brute_strip<8, 3, 3, true, false>;
        R = 8;
    } else if (fp.rho <= 4 && fp.n <= 4) {
        k = brute_strip<8, 4, 4, false, false>;
        R = 8;
    } else if (fp.rho == 16 && fp.n == 3) {
        k = brute_strip<8, 16, 3, true, false>;
        R = 8;
    } else if (fp.rho <= 16 && fp.n <= 16) {
        k = brute_strip<2, 16, 16, false, false>;
        R = 2;
    } else if (fp.rho == 32 && fp.n == 32 && same) {
        k = brute_strip<2, 32, 32, true, true>;
        R = 2;
    } else if (fp.rho <= 32 && fp.n <= 32) {
        k = brute_strip<1, 32, 32, false, false>;
        R = 1;
    } else {
        k = brute_strip<1, FHD_MAX_RHO, FHD_MAX_N, false, false>;
        R = 1;
    }
    const int rows = R * (RT / 64);
    const dim3 g((fp.W + 63) / 64, (fp.H + rows - 1) / rows);
    hipEvent_t tb = c.stage_begin();
    hipLaunchKernelGGL(k, g, dim3(RT), 0, c.stream, a);
    c.stage_end(FHD_STAGE_BRUTE, tb);
    FHD_HIP(hipGetLastError());
}


size_t approx_error_workspace(int H, int W, int K, int rho) {
    const size_t blocks = (size_t)((W + AE_X - 1) / AE_X) * ((H + AE_Y - 1) / AE_Y);
    return align_up(sizeof(double) * (blocks + 1), 256) + align_up(filter_consts_bytes(K, rho), 256) + 512;
}

void approx_error_run(Ctx& c, Arena& ws, const float* guide, int rho, int H, int W, const float* centers_host,
                      const float* Pfp32_host, int K, int S, float sigma_r, float* err, double* mean) {
    FHD_REQUIRE(K >= 1 && K <= 64, FHD_EUNSUPPORTED, "the approximation error takes at most 64 clusters");
    const int RM = rho <= 4 ? 4 : (rho <= 16 ? 16 : 64);
    const size_t lds = approx_error_lds(K, RM);
    const size_t cb = filter_consts_bytes(K, rho);
    char* dev = ws.take<char>(cb);
    char* hs = static_cast<char*>(c.host_stage(1, cb));
    filter_consts_fill(centers_host, Pfp32_host, K, rho, hs);
    FHD_HIP(hipMemcpyAsync(dev, hs, cb, hipMemcpyHostToDevice, c.stream));
    c.stage_done(1);
    const FilterConsts kc = filter_consts_at(dev, K, rho);
    const int gx = (W + AE_X - 1) / AE_X;
    const int blocks = gx * ((H + AE_Y - 1) / AE_Y);
    double* part = ws.take<double>((size_t)blocks + 1);
    const float inv2s2 = std::isinf(sigma_r) ? 0.0f : (float)(1.0 / (2.0 * (double)sigma_r * sigma_r));
    auto launch = [&](auto kern) {
        FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(AE_T), lds, c.stream, guide, rho, H, W, K, S, inv2s2,
                           kc.mu, kc.P, err, gx, part);
    };
    if (RM == 4) launch(approx_error_kernel<4>);
    else if (RM == 16) launch(approx_error_kernel<16>);
    else launch(approx_error_kernel<64>);
    FHD_HIP(hipGetLastError());
    if (mean != nullptr) {
        sum_doubles(c, part, blocks, part + blocks);
        double* hm = static_cast<double*>(c.host_stage(2, sizeof(double)));
        FHD_HIP(hipMemcpyAsync(hm, part + blocks, sizeof(double), hipMemcpyDeviceToHost, c.stream));
        c.stage_done(2);
        FHD_HIP(hipStreamSynchronize(c.stream));
        *mean = *hm / ((double)H * W);
    }
}


size_t filter_volume_workspace(const FilterPlan& fp) {
    Arena probe;
    const size_t Np = (size_t)fp.H * fp.Wp;
    probe.take<char>(filter_consts_bytes(fp.K, fp.rho));
    probe.take<float>((size_t)fp.K * Np);
    probe.take<float>((size_t)fp.K * Np);
    probe.take<float>((size_t)fp.K * (fp.n + 1) * Np);
    probe.take<float>((size_t)fp.K * (fp.n + 1) * Np);
    return probe.used + 256;
}

void filter_volume_run(Ctx& c, Arena& ws, const FilterPlan& fp, int D, const float* f, const float* guide,
                       const float* centers_host, const float* Pfp32_host, const int* labels, float* out,
                       float* den) {
    FHD_REQUIRE(fp.H % D == 0, FHD_EINVAL, "internal: volume rows");
    const bool hard = fp.coef == FHD_COEF_HARD;
    FHD_REQUIRE(!hard || labels != nullptr, FHD_EINVAL, "internal: the hard variant needs labels");
    const int Hs = fp.H / D;
    const size_t cb = filter_consts_bytes(fp.K, fp.rho);
    char* dev = ws.take<char>(cb);
    char* hs = static_cast<char*>(c.host_stage(1, cb));
    filter_consts_fill(centers_host, Pfp32_host, fp.K, fp.rho, hs);
    FHD_HIP(hipMemcpyAsync(dev, hs, cb, hipMemcpyHostToDevice, c.stream));
    c.stage_done(1);
    const FilterConsts kc = filter_consts_at(dev, fp.K, fp.rho);
    const long long Np = (long long)fp.H * fp.Wp;
    float* Bpl = ws.take<float>((size_t)fp.K * Np);
    float* Cpl = ws.take<float>((size_t)fp.K * Np);
    float* pa = ws.take<float>((size_t)fp.K * (fp.n + 1) * Np);
    float* pb = ws.take<float>((size_t)fp.K * (fp.n + 1) * Np);
    FA a = make_args(fp);
    a.f = f;
    a.p = guide;
    a.mu = kc.mu;
    a.P = kc.P;
    a.out = out;
    a.den = den;
    a.labels = labels;
    a.Pp = Np;  // no halo rows
    hipStream_t st = c.stream;
    const int npx = weights_fp32_npx(fp.K);
    const size_t lds = weights_fp32_lds(fp.K, fp.rho, npx);
    FHD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(weights_fp32),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipEvent_t tw = c.stage_begin();
    hipLaunchKernelGGL(weights_fp32, dim3((fp.W + npx - 1) / npx, fp.H), dim3(npx), lds, st, a, Bpl,
                       hard ? nullptr : Cpl);
    c.stage_end(FHD_STAGE_WEIGHTS, tw);
    FHD_HIP(hipGetLastError());
    a.Bpl = Bpl;
    a.Cpl = Cpl;
    const long long planes = (long long)fp.K * (fp.n + 1);
    auto grid = [](long long threads) { return dim3((unsigned)((threads + RT - 1) / RT)); };
    hipEvent_t tr = c.stage_begin();
    // the convolved factor: c_l [f, 1] (least squares, transposed form) or
    // b_l [f, 1] (hard variant, eqs. (17)-(18))
    hipLaunchKernelGGL(vol_fir_x, grid((long long)fp.K * fp.N), dim3(RT), 0, st, a, hard ? Bpl : Cpl, pa);
    c.stage_end(FHD_STAGE_ROW, tr);
    hipEvent_t tc = c.stage_begin();
    hipLaunchKernelGGL(vol_fir_yz, grid(planes * D * ((Hs + VR - 1) / VR) * fp.W), dim3(RT), 0, st, a, D, Hs, 1, pa,
                       pb);
    hipLaunchKernelGGL(vol_fir_yz, grid(planes * Hs * ((D + VR - 1) / VR) * fp.W), dim3(RT), 0, st, a, D, Hs, 2, pb,
                       pa);
    a.planes = pa;
    hipLaunchKernelGGL(recomb_young, dim3((unsigned)((fp.N + RT - 1) / RT)), dim3(RT), 0, st, a, hard ? 1 : 0);
    c.stage_end(FHD_STAGE_COL, tc);
    FHD_HIP(hipGetLastError());
}

void bruteforce_volume_run(Ctx& c, const FilterPlan& fp, int D, const float* f, const float* guide, float* out,
                           float* den) {
    FHD_REQUIRE(fp.H % D == 0, FHD_EINVAL, "internal: volume rows");
    FA a = make_args(fp);
    a.f = f;
    a.p = guide;
    hipEvent_t tb = c.stage_begin();
    hipLaunchKernelGGL(brute_volume, dim3((unsigned)((fp.N + RT - 1) / RT)), dim3(RT), 0, c.stream, a, D, fp.H / D,
                       out, den);
    c.stage_end(FHD_STAGE_BRUTE, tb);
    FHD_HIP(hipGetLastError());
}
}  // namespace fhd
