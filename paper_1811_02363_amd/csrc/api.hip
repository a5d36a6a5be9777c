// The C ABI of include/fhd.h: argument checks, workspace, orchestration of
// the steps of Algorithm 1, and conversion of failures into status codes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <atomic>
#include <exception>
#include <mutex>
#include <new>
#include <thread>
#include <string>
#include <vector>

#include "fhd_internal.h"

// Scratch of fhd_filter_centers_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never uses its name as an
// address: each device's copy is looked up once with hipGetSymbolAddress
// (fhd::noalloc_scratch_address) and that pointer is what kernels receive.
static __device__ __align__(256) char scratch[FHD_NOALLOC_SCRATCH_BYTES];

namespace fhd {

Arena Ctx::arena(size_t need) {
    Arena a;
    if (ext_ws != nullptr) {
        FHD_REQUIRE(need <= ext_bytes, FHD_ENOMEM, "caller workspace too small");
        a.base = static_cast<char*>(ext_ws);
        a.cap = ext_bytes;
        return a;
    }
    if (own_bytes < need) {
        if (own_ws != nullptr) {
            FHD_HIP(hipStreamSynchronize(stream));
            FHD_HIP(hipFree(own_ws));
            own_ws = nullptr;
            own_bytes = 0;
        }
        const size_t bytes = align_up(need + need / 8, 1 << 20);
        if (hipMalloc(&own_ws, bytes) != hipSuccess) {
            own_ws = nullptr;
            (void)hipGetLastError();
            throw Error(FHD_ENOMEM, "device workspace allocation failed");
        }
        own_bytes = bytes;
    }
    a.base = static_cast<char*>(own_ws);
    a.cap = own_bytes;
    return a;
}

void* Ctx::host_stage(int slot, size_t bytes) {
    if (pinned_pending[slot]) {
        FHD_HIP(hipEventSynchronize(pinned_ev[slot]));
        pinned_pending[slot] = false;
    }
    if (pinned_bytes[slot] < bytes) {
        if (pinned[slot] != nullptr) FHD_HIP(hipHostFree(pinned[slot]));
        pinned[slot] = nullptr;
        pinned_bytes[slot] = 0;
        const size_t b = align_up(std::max<size_t>(bytes, 1 << 16), 1 << 16);
        if (hipHostMalloc(&pinned[slot], b, hipHostMallocDefault) != hipSuccess) {
            pinned[slot] = nullptr;
            (void)hipGetLastError();
            throw Error(FHD_ENOMEM, "pinned host allocation failed");
        }
        pinned_bytes[slot] = b;
    }
    if (pinned_ev[slot] == nullptr) FHD_HIP(hipEventCreateWithFlags(&pinned_ev[slot], hipEventDisableTiming));
    return pinned[slot];
}

void Ctx::stage_done(int slot) {
    FHD_HIP(hipEventRecord(pinned_ev[slot], stream));
    pinned_pending[slot] = true;
}

hipEvent_t Ctx::take_event() {
    if (!ev_pool.empty()) {
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    FHD_HIP(hipEventCreate(&e));
    return e;
}

hipEvent_t Ctx::stage_begin() {
    if (!timing) return nullptr;
    hipEvent_t e = take_event();
    FHD_HIP(hipEventRecord(e, stream));
    return e;
}

void Ctx::stage_end(int stage, hipEvent_t begin, int launches) {
    if (!timing || begin == nullptr) return;
    hipEvent_t e = take_event();
    FHD_HIP(hipEventRecord(e, stream));
    ev_rec[stage].push_back(EvPair{begin, e, launches});
}

void Ctx::fork(int n) {
    for (int k = 0; k <= NAUX; ++k)
        if (aux_ev[k] == nullptr) FHD_HIP(hipEventCreateWithFlags(&aux_ev[k], hipEventDisableTiming));
    for (int k = 0; k < n; ++k)
        if (aux[k] == nullptr) FHD_HIP(hipStreamCreateWithFlags(&aux[k], hipStreamNonBlocking));
    FHD_HIP(hipEventRecord(aux_ev[NAUX], stream));
    for (int k = 0; k < n; ++k) FHD_HIP(hipStreamWaitEvent(aux[k], aux_ev[NAUX], 0));
}

void Ctx::join(int n) {
    for (int k = 0; k < n; ++k) {
        FHD_HIP(hipEventRecord(aux_ev[k], aux[k]));
        FHD_HIP(hipStreamWaitEvent(stream, aux_ev[k], 0));
    }
}

void Ctx::release() {
    for (int k = 0; k < NAUX; ++k)
        if (aux[k] != nullptr) {
            (void)hipStreamSynchronize(aux[k]);
            (void)hipStreamDestroy(aux[k]);
            aux[k] = nullptr;
        }
    for (int k = 0; k <= NAUX; ++k)
        if (aux_ev[k] != nullptr) {
            (void)hipEventDestroy(aux_ev[k]);
            aux_ev[k] = nullptr;
        }
    (void)hipStreamSynchronize(stream);
    if (own_ws != nullptr) (void)hipFree(own_ws);
    own_ws = nullptr;
    for (auto& v : ev_rec)
        for (auto& pr : v) {
            ev_pool.push_back(pr.begin);
            ev_pool.push_back(pr.end);
        }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    ev_pool.clear();
    if (switch_ev != nullptr) (void)hipEventDestroy(switch_ev);
    switch_ev = nullptr;
    if (noalloc_ev != nullptr) (void)hipEventDestroy(noalloc_ev);
    noalloc_ev = nullptr;
    if (noalloc_pinned != nullptr) (void)hipHostFree(noalloc_pinned);
    noalloc_pinned = nullptr;
    noalloc_scratch = nullptr;
    for (int s = 0; s < 3; ++s) {
        if (pinned[s] != nullptr) (void)hipHostFree(pinned[s]);
        if (pinned_ev[s] != nullptr) (void)hipEventDestroy(pinned_ev[s]);
        pinned[s] = nullptr;
        pinned_ev[s] = nullptr;
    }
}

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) FHD_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int resolve_radius(const fhd_params& p) {
    if (p.spatial == FHD_SPATIAL_YOUNG) return 0;  // infinite support, no window radius
    if (p.radius >= 0) return p.radius;
    return (int)std::ceil(3.0 * (double)p.sigma_s - 1e-9);
}

void check_params(const fhd_params* p, int n, int rho, int H, int W) {
    FHD_REQUIRE(p != nullptr, FHD_EINVAL, "params is NULL");
    FHD_REQUIRE(n >= 1 && rho >= 1 && H >= 1 && W >= 1, FHD_EINVAL, "n, rho, H, W must be >= 1");
    FHD_REQUIRE(n <= FHD_MAX_N, FHD_EUNSUPPORTED, "n exceeds FHD_MAX_N");
    FHD_REQUIRE(rho <= FHD_MAX_RHO, FHD_EUNSUPPORTED, "rho exceeds FHD_MAX_RHO");
    FHD_REQUIRE((long long)H * W < (1LL << 31), FHD_EUNSUPPORTED, "image has 2^31 pixels or more");
    FHD_REQUIRE(p->spatial == FHD_SPATIAL_GAUSSIAN || p->spatial == FHD_SPATIAL_BOX ||
                    p->spatial == FHD_SPATIAL_YOUNG,
                FHD_EINVAL, "unknown spatial kernel");
    if (p->spatial == FHD_SPATIAL_GAUSSIAN)
        FHD_REQUIRE(p->sigma_s > 0.0f && std::isfinite(p->sigma_s), FHD_EINVAL, "sigma_s must be > 0");
    else if (p->spatial == FHD_SPATIAL_YOUNG)
        FHD_REQUIRE(p->sigma_s >= 0.5f && std::isfinite(p->sigma_s), FHD_EINVAL,
                    "the recursive Gaussian needs sigma_s >= 0.5");
    else
        FHD_REQUIRE(p->radius >= 0, FHD_EINVAL, "the box kernel needs radius >= 0");
    FHD_REQUIRE(p->sigma_r > 0.0f && !std::isnan(p->sigma_r), FHD_EINVAL, "sigma_r must be > 0");
    FHD_REQUIRE(p->K >= 1 && p->K <= FHD_MAX_K, FHD_EINVAL, "K must be in [1, FHD_MAX_K]");
    FHD_REQUIRE((long long)p->K <= (long long)H * W, FHD_EINVAL, "K exceeds the number of pixels");
    FHD_REQUIRE(p->coef == FHD_COEF_LSQ || p->coef == FHD_COEF_HARD || p->coef == FHD_COEF_EXACT, FHD_EINVAL,
                "unknown coef");
    FHD_REQUIRE(p->contract == FHD_CONTRACT_FP32 || p->contract == FHD_CONTRACT_BF16 ||
                    p->contract == FHD_CONTRACT_FP16,
                FHD_EINVAL, "unknown contraction precision");
    FHD_REQUIRE(p->kmeans_max_iter >= 1, FHD_EINVAL, "kmeans_max_iter must be >= 1");
    const int S = resolve_radius(*p);
    FHD_REQUIRE(S >= 0 && S <= FHD_MAX_RADIUS, FHD_EUNSUPPORTED, "radius exceeds FHD_MAX_RADIUS");
}

FilterPlan make_plan(const fhd_params& p, int n, int rho, int H, int W, int K) {
    FilterPlan fp{};
    fp.n = n;
    fp.rho = rho;
    fp.H = H;
    fp.W = W;
    fp.K = K;
    fp.S = resolve_radius(p);
    fp.spatial = p.spatial;
    fp.contract = p.contract;
    fp.coef = p.coef;
    fp.sigma_s = p.sigma_s;
    fp.sigma_r = p.sigma_r;
    fp.N = (long long)H * W;
    fp.Wp = (int)align_up((size_t)W, 32);  // plane rows start on 128-byte lines
    fp.materialize = rho > 8 || K > 32 || p.contract != FHD_CONTRACT_FP32 || p.spatial == FHD_SPATIAL_YOUNG ||
                     p.coef == FHD_COEF_EXACT;
    return fp;
}

// The per-pixel fit of eq. (10) as the filter's coefficients: the forms the
// kernel covers, and only the calls that take it.
void check_exact(const fhd_params* p, int K) {
    if (p->coef != FHD_COEF_EXACT) return;
    FHD_REQUIRE(K <= EXACT_LS_MAX_K, FHD_EUNSUPPORTED, "coefficients from eq. (10) take K <= 32");
    FHD_REQUIRE(p->contract == FHD_CONTRACT_FP32, FHD_EUNSUPPORTED, "coefficients from eq. (10) take the FP32 form");
    FHD_REQUIRE(p->spatial != FHD_SPATIAL_YOUNG, FHD_EUNSUPPORTED,
                "coefficients from eq. (10) need a finite window (Gaussian or box)");
}

void reject_exact(const fhd_params* p, const char* call) {
    FHD_REQUIRE(p->coef != FHD_COEF_EXACT, FHD_EUNSUPPORTED,
                std::string(call) + " does not take coefficients from eq. (10) (fhd_filter, fhd_filter_centers do)");
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    if (a == nullptr || b == nullptr) return false;
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + nb && y < x + na;
}

// The K x K solve on FP32 centers: A, A^+ (FP64) and its FP32 copy.
PinvResult solve(const float* centers, int K, int rho, double sigma_r, double rtol, std::vector<float>& P32) {
    std::vector<double> A((size_t)K * K), P((size_t)K * K);
    kernel_matrix(centers, K, rho, sigma_r, A.data());
    PinvResult r = pinv_symmetric(A.data(), K, rtol, P.data());
    P32.resize((size_t)K * K);
    for (size_t q = 0; q < P.size(); ++q) P32[q] = (float)P[q];
    return r;
}

template <class F>
fhd_status guarded(fhd_ctx* ctx, F&& body) {
    if (ctx == nullptr) return FHD_EINVAL;
    ctx->impl.err.clear();
    try {
        DeviceGuard g(ctx->impl.device);
        body(ctx->impl);
        return FHD_OK;
    } catch (const Error& e) {
        ctx->impl.err = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        ctx->impl.err = "host allocation failed";
        return FHD_ENOMEM;
    } catch (const std::exception& e) {
        ctx->impl.err = e.what();
        return FHD_EINVAL;
    } catch (...) {
        ctx->impl.err = "unknown failure";
        return FHD_EINVAL;
    }
}

// out[d][i] = guide[d][i] / sigma_d, correctly rounded; one thread per entry.
struct RangeScales {
    float s[FHD_MAX_RHO];
};
__global__ __launch_bounds__(256) void scale_guide_kernel(const float* guide, long long N, int rho, RangeScales sc,
                                                          float* out) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * rho) return;
    out[e] = __fdiv_rn(guide[e], sc.s[(int)(e / N)]);
}

// Diagnostics of the normaliser r_hat of eq. (16) and of the output (the
// least-squares coefficients may be negative, so r_hat can come out tiny or
// non-positive; the ratio is not guarded): per block, the smallest r_hat and
// the counts of r_hat <= 0 (or NaN), r_hat < 1e-3 and non-finite outputs.
// The blocks' records are reduced on the host in a fixed order.
constexpr int STAT_T = 256, STAT_BLOCKS = 512;
struct StatRec {
    float dmin;
    unsigned pad;
    unsigned long long nonpos, small, nonfinite;
};
struct OutStats {
    float den_min = INFINITY;
    long long nonpos = 0, small = 0, nonfinite = 0;
};

__global__ __launch_bounds__(STAT_T) void out_stats_kernel(const float* __restrict__ out, long long count,
                                                           const float* __restrict__ den, long long N,
                                                           StatRec* __restrict__ part) {
    float mn = INFINITY;
    unsigned long long np = 0, sm = 0, nf = 0;
    const long long stride = (long long)gridDim.x * STAT_T;
    const long long i0 = (long long)blockIdx.x * STAT_T + threadIdx.x;
    if (den != nullptr)
        for (long long i = i0; i < N; i += stride) {
            const float d = den[i];
            mn = fminf(mn, d);
            np += !(d > 0.0f);
            sm += !(d >= 1e-3f);
        }
    for (long long i = i0; i < count; i += stride) nf += !isfinite(out[i]);
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o));
        np += __shfl_xor(np, o);
        sm += __shfl_xor(sm, o);
        nf += __shfl_xor(nf, o);
    }
    __shared__ StatRec w[STAT_T / 64];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) w[wave] = StatRec{mn, 0u, np, sm, nf};
    __syncthreads();
    if (threadIdx.x == 0) {
        StatRec r = w[0];
        for (int q = 1; q < STAT_T / 64; ++q) {
            r.dmin = fminf(r.dmin, w[q].dmin);
            r.nonpos += w[q].nonpos;
            r.small += w[q].small;
            r.nonfinite += w[q].nonfinite;
        }
        part[blockIdx.x] = r;
    }
}

size_t stats_workspace(long long N) {
    return align_up(sizeof(float) * (size_t)N, 256) + align_up(sizeof(StatRec) * STAT_BLOCKS, 256);
}

// Enqueues the statistics of `count` outputs and N normalisers (den may be
// null: outputs only) into a block of STAT_BLOCKS records.
void out_stats_launch(Ctx& c, const float* out, long long count, const float* den, long long N, StatRec* part) {
    hipLaunchKernelGGL(out_stats_kernel, dim3(STAT_BLOCKS), dim3(STAT_T), 0, c.stream, out, count, den, N, part);
    FHD_HIP(hipGetLastError());
}

OutStats out_stats_reduce(const StatRec* h) {
    OutStats s;
    for (int b = 0; b < STAT_BLOCKS; ++b) {
        s.den_min = std::fmin(s.den_min, h[b].dmin);
        s.nonpos += (long long)h[b].nonpos;
        s.small += (long long)h[b].small;
        s.nonfinite += (long long)h[b].nonfinite;
    }
    return s;
}

// One image's statistics; synchronises the stream.
OutStats out_stats(Ctx& c, Arena& ws, const float* out, long long count, const float* den, long long N) {
    StatRec* part = ws.take<StatRec>(STAT_BLOCKS);
    out_stats_launch(c, out, count, den, N, part);
    std::vector<StatRec> h(STAT_BLOCKS);
    FHD_HIP(hipMemcpyAsync(h.data(), part, sizeof(StatRec) * STAT_BLOCKS, hipMemcpyDeviceToHost, c.stream));
    FHD_HIP(hipStreamSynchronize(c.stream));
    return out_stats_reduce(h.data());
}

void strict_verdict(const OutStats& s) {
    FHD_REQUIRE(s.nonpos == 0 && s.nonfinite == 0, FHD_ENUMERIC,
                "non-positive normaliser (" + std::to_string(s.nonpos) + " pixels) or non-finite output (" +
                    std::to_string(s.nonfinite) + " values)");
}

void fill_stats(fhd_info* info, const OutStats& s) {
    if (info == nullptr) return;
    info->den_min = s.den_min;
    info->den_nonpos = s.nonpos;
    info->den_small = s.small;
    info->nonfinite = s.nonfinite;
}

void fill_info(fhd_info* info, int K_eff, const PinvResult& pr, double E_K, int rounds, int splits,
               double ms_cluster, double ms_solve, double ms_filter) {
    if (info == nullptr) return;
    std::memset(info, 0, sizeof(*info));
    info->K_eff = K_eff;
    info->pinv_rank = pr.rank;
    info->kmeans_rounds = rounds;
    info->kmeans_splits = splits;
    info->E_K = E_K;
    info->cond_A = pr.cond;
    info->pinv_norm = pr.max_abs;
    info->ms_cluster = (float)ms_cluster;
    info->ms_solve = (float)ms_solve;
    info->ms_filter = (float)ms_filter;
}

// body(i) for i in [0, n) on up to eight host threads (the per-image K x K
// solves of a batch); the first exception is rethrown after all have ended.
template <class F>
void parallel_for(int n, F&& body) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::min<int>(n, (int)std::min(8u, hw));
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) body(i);
        return;
    }
    std::atomic<int> next{0};
    std::exception_ptr err;
    std::mutex m;
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (;;) {
                const int i = next.fetch_add(1);
                if (i >= n) break;
                try {
                    body(i);
                } catch (...) {
                    std::lock_guard<std::mutex> g(m);
                    if (!err) err = std::current_exception();
                }
            }
        });
    for (auto& x : th) x.join();
    if (err) std::rethrow_exception(err);
}

// Per-image work of a batch spread over the auxiliary streams: while alive,
// `on(i)` points the context at stream i % n; the destructor joins the
// auxiliary streams back into the context's stream (also on errors).
struct Spread {
    Ctx& c;
    hipStream_t main;
    int n;
    Spread(Ctx& cx, int images) : c(cx), main(cx.stream), n(std::min(images, Ctx::NAUX)) { c.fork(n); }
    int on(int i) {
        c.stream = c.aux[i % n];
        return i % n;
    }
    ~Spread() {
        c.stream = main;
        try {
            c.join(n);
        } catch (...) {
        }
    }
};

// images by decreasing pixel count (ties by index): the order in which
// they are dealt to the streams
std::vector<int> by_size(const std::vector<long long>& cnt) {
    std::vector<int> o(cnt.size());
    for (size_t i = 0; i < o.size(); ++i) o[i] = (int)i;
    std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return cnt[x] > cnt[y]; });
    return o;
}

// Validates a ragged batch and returns the pixel count of every image; the
// images must be packed back to back (px_offset[0] = 0, each image right after
// the previous one).
std::vector<long long> batch_counts(int B, const int* H, const int* W, const long long* px_offset) {
    FHD_REQUIRE(B >= 1 && H != nullptr && W != nullptr && px_offset != nullptr, FHD_EINVAL,
                "batch needs B >= 1 and the H, W, px_offset arrays");
    std::vector<long long> cnt(B);
    long long next = 0;
    for (int b = 0; b < B; ++b) {
        FHD_REQUIRE(H[b] >= 1 && W[b] >= 1, FHD_EINVAL, "every image needs H, W >= 1");
        FHD_REQUIRE(px_offset[b] == next, FHD_EINVAL, "images must be packed back to back from offset 0");
        cnt[b] = (long long)H[b] * W[b];
        next += cnt[b];
    }
    FHD_REQUIRE(next < (1LL << 31), FHD_EUNSUPPORTED, "batch has 2^31 pixels or more");
    return cnt;
}

// ---- intermediates saved by a forward call for its adjoint ------------------

// The forward call's requirements on a saved buffer: the adjoint's window,
// FP32 contraction, least-squares coefficients, K <= 64.
void saved_check_ptr(const void* saved) {
    FHD_REQUIRE((reinterpret_cast<uintptr_t>(saved) & 255) == 0, FHD_EINVAL, "saved buffer must be 256-byte aligned");
}

void saved_check_params(const fhd_params* p, int K) {
    FHD_REQUIRE(p->contract == FHD_CONTRACT_FP32, FHD_EUNSUPPORTED,
                "saving for the adjoint needs the FP32 contraction (the adjoint differentiates it)");
    FHD_REQUIRE(p->coef == FHD_COEF_LSQ, FHD_EUNSUPPORTED, "saving for the adjoint needs least-squares coefficients");
    FHD_REQUIRE(p->spatial == FHD_SPATIAL_GAUSSIAN || p->spatial == FHD_SPATIAL_BOX, FHD_EUNSUPPORTED,
                "saving for the adjoint needs the truncated Gaussian or box window");
    const int S = resolve_radius(*p);
    FHD_REQUIRE(S >= 1 && S <= 32, FHD_EUNSUPPORTED, "saving for the adjoint needs radius 1..32");
    FHD_REQUIRE(K <= 64, FHD_EUNSUPPORTED, "saving for the adjoint needs K <= 64");
}

// the forward plan whose layout the saved buffer follows (FP32 contraction)
FilterPlan saved_plan(const fhd_params& p, int n, int rho, int H, int W, int K) {
    return make_plan(p, n, rho, H, W, K);
}

// byte offsets of the images' regions in a batch's saved buffer (sized with
// the requested K, so forward and adjoint agree before K_eff is known)
std::vector<size_t> saved_offsets(const fhd_params& p, int B, const int* H, const int* W, int n, int rho) {
    std::vector<size_t> off(B + 1, 0);
    for (int b = 0; b < B; ++b)
        off[b + 1] = off[b] + align_up(saved_planes_bytes(saved_plan(p, n, rho, H[b], W[b], p.K)), 256);
    return off;
}

Ctx::SavedDesc saved_desc(const void* ptr, size_t bytes, const float* f, const float* guide, int n, int rho,
                          const fhd_params& p) {
    Ctx::SavedDesc d;
    d.ptr = ptr;
    d.bytes = bytes;
    d.f = f;
    d.guide = guide;
    d.n = n;
    d.rho = rho;
    d.K = p.K;
    d.S = resolve_radius(p);
    d.spatial = p.spatial;
    d.sigma_s = p.spatial == FHD_SPATIAL_BOX ? 0.0f : p.sigma_s;  // the box ignores it
    d.sigma_r = p.sigma_r;
    d.rtol = p.pinv_rtol;
    return d;
}

void saved_register(Ctx& c, Ctx::SavedDesc d) {
    const char* lo = static_cast<const char*>(d.ptr);
    const char* hi = lo + d.bytes;
    auto& v = c.saved;
    v.erase(std::remove_if(v.begin(), v.end(),
                           [&](const Ctx::SavedDesc& e) {
                               const char* a = static_cast<const char*>(e.ptr);
                               return a < hi && lo < a + e.bytes;  // overwritten
                           }),
            v.end());
    v.push_back(std::move(d));
    if (v.size() > 16) v.erase(v.begin());
}

void saved_verify(const Ctx& c, const Ctx::SavedDesc& want) {
    for (auto it = c.saved.rbegin(); it != c.saved.rend(); ++it) {
        if (it->ptr != want.ptr) continue;
        const Ctx::SavedDesc& d = *it;
        FHD_REQUIRE(d.f == want.f && d.guide == want.guide && d.n == want.n && d.rho == want.rho &&
                        d.K == want.K && d.S == want.S && d.spatial == want.spatial && d.sigma_s == want.sigma_s &&
                        d.sigma_r == want.sigma_r && d.rtol == want.rtol && d.H == want.H && d.W == want.W &&
                        d.Keff == want.Keff && d.centers == want.centers,
                    FHD_EINVAL,
                    "saved buffer was written by a forward call with other arguments (image, guide, shape, "
                    "window, sigmas or centers)");
        FHD_REQUIRE(want.bytes <= d.bytes, FHD_EINVAL, "saved buffer smaller than the forward call's");
        return;
    }
    throw Error(FHD_EINVAL, "saved buffer was not written by a forward call on this context (or was overwritten since)");
}

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mutex;
char* noalloc_addr[NOALLOC_MAX_DEVICES] = {};

// The address of `scratch` on `device` (which must be the current device).
char* noalloc_scratch_address(int device) {
    FHD_REQUIRE(device >= 0 && device < NOALLOC_MAX_DEVICES, FHD_EUNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> g(noalloc_mutex);
    if (noalloc_addr[device] == nullptr) {
        void* ptr = nullptr;
        FHD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        FHD_REQUIRE(ptr != nullptr && (reinterpret_cast<uintptr_t>(ptr) & 255) == 0, FHD_EHIP,
                    "static scratch has no usable device address");
        noalloc_addr[device] = static_cast<char*>(ptr);
    }
    return noalloc_addr[device];
}

}  // namespace
}  // namespace fhd

using namespace fhd;

extern "C" {

void fhd_default_params(fhd_params* p) {
    if (p == nullptr) return;
    std::memset(p, 0, sizeof(*p));
    p->sigma_s = 3.0f;
    p->radius = -1;
    p->sigma_r = 0.1f;
    p->K = 16;
    p->spatial = FHD_SPATIAL_GAUSSIAN;
    p->contract = FHD_CONTRACT_FP32;
    p->coef = FHD_COEF_LSQ;
    p->kmeans_max_iter = 20;
    p->pinv_rtol = 0.0;
    p->strict = 0;
}

fhd_status fhd_create(fhd_ctx** out, int device, void* hip_stream) {
    if (out == nullptr) return FHD_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return device < 0 ? FHD_EINVAL : FHD_EHIP;
    }
    fhd_ctx* c = new (std::nothrow) fhd_ctx();
    if (c == nullptr) return FHD_ENOMEM;
    c->impl.device = device;
    c->impl.stream = static_cast<hipStream_t>(hip_stream);
    // set-up of the allocation-free entry point on this device: the static
    // scratch's address and the pinned constants buffer
    const fhd_status st = guarded(c, [&](Ctx& x) {
        x.noalloc_scratch = noalloc_scratch_address(device);
        const size_t cb = filter_consts_bytes(FHD_MAX_K, FHD_MAX_RHO);
        if (hipHostMalloc(&x.noalloc_pinned, cb, hipHostMallocDefault) != hipSuccess) {
            x.noalloc_pinned = nullptr;
            (void)hipGetLastError();
            throw Error(FHD_ENOMEM, "pinned host allocation failed");
        }
        FHD_HIP(hipEventCreateWithFlags(&x.noalloc_ev, hipEventDisableTiming));
    });
    if (st != FHD_OK) {
        fhd_destroy(c);
        return st;
    }
    *out = c;
    return FHD_OK;
}

fhd_status fhd_destroy(fhd_ctx* ctx) {
    if (ctx == nullptr) return FHD_EINVAL;
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(ctx->impl.device);
        ctx->impl.release();
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    delete ctx;
    return FHD_OK;
}

fhd_status fhd_set_stream(fhd_ctx* ctx, void* hip_stream) {
    return guarded(ctx, [&](Ctx& c) {
        // the staging slots may still feed copies on the old stream
        for (int s = 0; s < 3; ++s)
            if (c.pinned_pending[s]) {
                FHD_HIP(hipEventSynchronize(c.pinned_ev[s]));
                c.pinned_pending[s] = false;
            }
        hipStream_t ns = static_cast<hipStream_t>(hip_stream);
        if (ns != c.stream) {
            // work already enqueued on the old stream still reads and writes
            // the context's workspace: the new stream starts after it
            if (c.switch_ev == nullptr)
                FHD_HIP(hipEventCreateWithFlags(&c.switch_ev, hipEventDisableTiming));
            FHD_HIP(hipEventRecord(c.switch_ev, c.stream));
            FHD_HIP(hipStreamWaitEvent(ns, c.switch_ev, 0));
        }
        c.stream = ns;
    });
}

const char* fhd_last_error(const fhd_ctx* ctx) {
    if (ctx == nullptr) return "context is NULL";
    return ctx->impl.err.c_str();
}

fhd_status fhd_workspace_size(const fhd_params* p, int n, int rho, int H, int W, size_t* bytes) {
    if (bytes == nullptr) return FHD_EINVAL;
    try {
        check_params(p, n, rho, H, W);
        const FilterPlan fp = make_plan(*p, n, rho, H, W, p->K);
        size_t b = kmeans_workspace(fp.N, rho, p->K);
        b += filter_workspace(fp);
        b += align_up(sizeof(int) * (size_t)fp.N, 256);  // labels
        b += stats_workspace(fp.N);                      // normaliser statistics (info, strict)
        b += 4096;                                       // slack
        *bytes = b;
        return FHD_OK;
    } catch (const Error& e) {
        return e.status;
    } catch (...) {
        return FHD_EINVAL;
    }
}

fhd_status fhd_saved_size(const fhd_params* p, int n, int rho, int H, int W, size_t* bytes) {
    if (bytes == nullptr) return FHD_EINVAL;
    try {
        check_params(p, n, rho, H, W);
        saved_check_params(p, p->K);
        *bytes = saved_planes_bytes(saved_plan(*p, n, rho, H, W, p->K));
        return FHD_OK;
    } catch (const Error& e) {
        return e.status;
    } catch (...) {
        return FHD_EINVAL;
    }
}

fhd_status fhd_saved_size_batch(const fhd_params* p, int B, const int* H, const int* W, int n, int rho,
                                size_t* bytes) {
    if (bytes == nullptr || H == nullptr || W == nullptr || B < 1) return FHD_EINVAL;
    try {
        for (int b = 0; b < B; ++b) check_params(p, n, rho, H[b], W[b]);
        saved_check_params(p, p->K);
        *bytes = saved_offsets(*p, B, H, W, n, rho)[B];
        return FHD_OK;
    } catch (const Error& e) {
        return e.status;
    } catch (...) {
        return FHD_EINVAL;
    }
}

fhd_status fhd_set_workspace(fhd_ctx* ctx, void* dev, size_t bytes) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(dev == nullptr || (reinterpret_cast<uintptr_t>(dev) & 255) == 0, FHD_EINVAL,
                    "workspace must be 256-byte aligned");
        FHD_HIP(hipStreamSynchronize(c.stream));
        c.ext_ws = dev;
        c.ext_bytes = dev ? bytes : 0;
    });
}

fhd_status fhd_cluster(fhd_ctx* ctx, const float* guide, int rho, int H, int W, int K, int max_iter,
                       float* centers, int* labels, int* K_eff, fhd_info* info) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(guide != nullptr && centers != nullptr, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(rho >= 1 && H >= 1 && W >= 1, FHD_EINVAL, "rho, H, W must be >= 1");
        FHD_REQUIRE(rho <= FHD_MAX_RHO, FHD_EUNSUPPORTED, "rho exceeds FHD_MAX_RHO");
        const long long N = (long long)H * W;
        FHD_REQUIRE(K >= 1 && K <= FHD_MAX_K && K <= N, FHD_EINVAL, "K out of range");
        Arena ws = c.arena(kmeans_workspace(N, rho, K));
        const auto t0 = clk::now();
        KmResult km;
        kmeans_run(c, ws, guide, rho, N, K, max_iter, labels, km);
        for (size_t q = 0; q < km.centers.size(); ++q) centers[q] = (float)km.centers[q];
        if (K_eff) *K_eff = km.K_eff;
        c.last_keff = km.K_eff;
        FHD_HIP(hipStreamSynchronize(c.stream));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->K_eff = km.K_eff;
            info->E_K = km.E_K;
            info->kmeans_rounds = km.rounds;
            info->kmeans_splits = km.splits;
            info->ms_cluster = (float)ms_since(t0);
        }
    });
}

fhd_status fhd_pinv(const float* centers, int K, int rho, double sigma_r, double rtol, double* A,
                    double* Apinv, int* rank, double* cond) {
    if (centers == nullptr || K < 1 || K > FHD_MAX_K || rho < 1 || rho > FHD_MAX_RHO || !(sigma_r > 0.0))
        return FHD_EINVAL;
    try {
        std::vector<double> a((size_t)K * K), p((size_t)K * K);
        kernel_matrix(centers, K, rho, sigma_r, a.data());
        const PinvResult r = pinv_symmetric(a.data(), K, rtol, p.data());
        if (A) std::memcpy(A, a.data(), sizeof(double) * a.size());
        if (Apinv) std::memcpy(Apinv, p.data(), sizeof(double) * p.size());
        if (rank) *rank = r.rank;
        if (cond) *cond = r.cond;
        return FHD_OK;
    } catch (const Error& e) {
        return e.status;
    } catch (...) {
        return FHD_ENOMEM;
    }
}

fhd_status fhd_filter_centers(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int H,
                              int W, const float* centers, int K, const int* labels, const fhd_params* p,
                              float* out, float* den, fhd_info* info, void* saved, size_t saved_bytes) {
    return guarded(ctx, [&](Ctx& c) {
        check_params(p, n, rho, H, W);
        FHD_REQUIRE(f && guide && centers && out, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(K >= 1 && K <= FHD_MAX_K, FHD_EINVAL, "K must be in [1, FHD_MAX_K]");
        FHD_REQUIRE(p->coef != FHD_COEF_HARD || labels != nullptr, FHD_EINVAL, "hard coefficients need labels");
        check_exact(p, K);
        const long long N = (long long)H * W;
        FHD_REQUIRE(!ranges_overlap(out, sizeof(float) * N * n, f, sizeof(float) * N * n) &&
                        !ranges_overlap(out, sizeof(float) * N * n, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, f, sizeof(float) * N * n) &&
                        !ranges_overlap(den, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, out, sizeof(float) * N * n),
                    FHD_EINVAL, "outputs alias inputs");
        const FilterPlan fp = make_plan(*p, n, rho, H, W, K);
        SavedPlanes sv{};
        if (saved != nullptr) {
            saved_check_ptr(saved);
            saved_check_params(p, K);
            FHD_REQUIRE(saved_bytes >= saved_planes_bytes(fp), FHD_EINVAL, "saved buffer too small (fhd_saved_size)");
            FHD_REQUIRE(!ranges_overlap(saved, saved_bytes, f, sizeof(float) * N * n) &&
                            !ranges_overlap(saved, saved_bytes, guide, sizeof(float) * N * rho) &&
                            !ranges_overlap(saved, saved_bytes, out, sizeof(float) * N * n) &&
                            !ranges_overlap(saved, saved_bytes, den, sizeof(float) * N),
                        FHD_EINVAL, "saved buffer aliases an input or output");
            sv = saved_at(static_cast<char*>(saved), fp);
        }
        Arena ws = c.arena(filter_workspace(fp) + stats_workspace(N) + 4096);
        const bool stats = info != nullptr || p->strict;
        float* dn = (stats && den == nullptr) ? ws.take<float>((size_t)N) : den;
        const auto t0 = clk::now();
        std::vector<float> P32;
        const PinvResult pr = solve(centers, K, rho, p->sigma_r, p->pinv_rtol, P32);
        const double ms_solve = ms_since(t0);
        const auto t1 = clk::now();
        filter_run(c, ws, fp, f, guide, centers, P32.data(), labels, out, dn, saved != nullptr ? &sv : nullptr);
        if (saved != nullptr) {
            Ctx::SavedDesc d = saved_desc(saved, saved_bytes, f, guide, n, rho, *p);
            d.K = K;
            d.H = {H};
            d.W = {W};
            d.Keff = {K};
            d.centers.assign(centers, centers + (size_t)K * rho);
            saved_register(c, std::move(d));
        }
        double ms_filter = 0.0;
        if (info) {
            FHD_HIP(hipStreamSynchronize(c.stream));
            ms_filter = ms_since(t1);
        }
        OutStats st;
        if (stats) st = out_stats(c, ws, out, N * n, dn, N);
        fill_info(info, K, pr, 0.0, 0, 0, 0.0, ms_solve, ms_filter);
        fill_stats(info, st);
        if (p->strict) strict_verdict(st);
    });
}

fhd_status fhd_filter_centers_noalloc(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int H,
                                      int W, const float* centers, int K, const int* labels, const fhd_params* p,
                                      float* out, float* den) {
    return guarded(ctx, [&](Ctx& c) {
        check_params(p, n, rho, H, W);
        FHD_REQUIRE(f && guide && centers && out, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(K >= 1 && K <= FHD_MAX_K, FHD_EINVAL, "K must be in [1, FHD_MAX_K]");
        FHD_REQUIRE(p->coef != FHD_COEF_HARD || labels != nullptr, FHD_EINVAL, "hard coefficients need labels");
        FHD_REQUIRE(c.noalloc_scratch != nullptr && c.noalloc_pinned != nullptr, FHD_EINVAL,
                    "context was not set up for the allocation-free call");
        reject_exact(p, "fhd_filter_centers_noalloc");
        const long long N = (long long)H * W;
        FHD_REQUIRE(!ranges_overlap(out, sizeof(float) * N * n, f, sizeof(float) * N * n) &&
                        !ranges_overlap(out, sizeof(float) * N * n, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, f, sizeof(float) * N * n) &&
                        !ranges_overlap(den, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, out, sizeof(float) * N * n),
                    FHD_EINVAL, "outputs alias inputs");
        const FilterPlan fp = make_plan(*p, n, rho, H, W, K);
        const size_t cb = filter_consts_bytes(K, rho);
        const size_t need = align_up(cb, 256) + filter_passes_workspace(fp) + (p->strict ? stats_workspace(N) : 0) + 1024;
        FHD_REQUIRE(need <= FHD_NOALLOC_SCRATCH_BYTES, FHD_ENOMEM,
                    "this image needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                        std::to_string((size_t)FHD_NOALLOC_SCRATCH_BYTES));
        Arena ws;
        ws.base = c.noalloc_scratch;
        ws.cap = FHD_NOALLOC_SCRATCH_BYTES;
        std::vector<float> P32;
        (void)solve(centers, K, rho, p->sigma_r, p->pinv_rtol, P32);
        // constants through the context's fixed pinned buffer, once the
        // previous copy out of it has ended
        if (c.noalloc_pending) {
            FHD_HIP(hipEventSynchronize(c.noalloc_ev));
            c.noalloc_pending = false;
        }
        char* dev = ws.take<char>(cb);
        filter_consts_fill(centers, P32.data(), K, rho, static_cast<char*>(c.noalloc_pinned));
        FHD_HIP(hipMemcpyAsync(dev, c.noalloc_pinned, cb, hipMemcpyHostToDevice, c.stream));
        FHD_HIP(hipEventRecord(c.noalloc_ev, c.stream));
        c.noalloc_pending = true;
        // stage timing would create events: off for this call
        const bool timing = c.timing;
        c.timing = false;
        try {
            float* dn = (p->strict && den == nullptr) ? ws.take<float>((size_t)N) : den;
            filter_passes(c, ws, fp, f, guide, filter_consts_at(dev, K, rho), labels, out, dn);
            if (p->strict) strict_verdict(out_stats(c, ws, out, N * n, dn, N));
        } catch (...) {
            c.timing = timing;
            throw;
        }
        c.timing = timing;
    });
}

fhd_status fhd_filter(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int H, int W,
                      const fhd_params* p, float* out, float* centers_out, float* den, fhd_info* info, void* saved,
                      size_t saved_bytes) {
    return guarded(ctx, [&](Ctx& c) {
        check_params(p, n, rho, H, W);
        check_exact(p, p->K);
        FHD_REQUIRE(f && guide && out, FHD_EINVAL, "NULL pointer");
        const long long N = (long long)H * W;
        FHD_REQUIRE(!ranges_overlap(out, sizeof(float) * N * n, f, sizeof(float) * N * n) &&
                        !ranges_overlap(out, sizeof(float) * N * n, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, f, sizeof(float) * N * n) &&
                        !ranges_overlap(den, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, out, sizeof(float) * N * n),
                    FHD_EINVAL, "outputs alias inputs");
        size_t need = 0;
        {
            const FilterPlan fp0 = make_plan(*p, n, rho, H, W, p->K);
            need = kmeans_workspace(N, rho, p->K) + filter_workspace(fp0) +
                   align_up(sizeof(int) * (size_t)N, 256) + stats_workspace(N) + 4096;
        }
        if (saved != nullptr) {
            saved_check_ptr(saved);
            saved_check_params(p, p->K);
            FHD_REQUIRE(saved_bytes >= saved_planes_bytes(make_plan(*p, n, rho, H, W, p->K)), FHD_EINVAL,
                        "saved buffer too small (fhd_saved_size)");
            FHD_REQUIRE(!ranges_overlap(saved, saved_bytes, f, sizeof(float) * N * n) &&
                            !ranges_overlap(saved, saved_bytes, guide, sizeof(float) * N * rho) &&
                            !ranges_overlap(saved, saved_bytes, out, sizeof(float) * N * n) &&
                            !ranges_overlap(saved, saved_bytes, den, sizeof(float) * N),
                        FHD_EINVAL, "saved buffer aliases an input or output");
        }
        Arena ws = c.arena(need);
        const bool hard = p->coef == FHD_COEF_HARD;
        int* labels = hard ? ws.take<int>((size_t)N) : nullptr;
        const bool stats = info != nullptr || p->strict;
        float* dn = (stats && den == nullptr) ? ws.take<float>((size_t)N) : den;
        const auto t0 = clk::now();
        KmResult km;
        {
            Arena kws = ws;  // the clustering scratch is dead once the centers are known
            kmeans_run(c, kws, guide, rho, N, p->K, p->kmeans_max_iter, labels, km);
        }
        const double ms_cluster = ms_since(t0);
        const int K = km.K_eff;
        c.last_keff = K;
        std::vector<float> c32((size_t)K * rho);
        for (size_t q = 0; q < c32.size(); ++q) c32[q] = (float)km.centers[q];
        if (centers_out) std::memcpy(centers_out, c32.data(), sizeof(float) * c32.size());
        const auto t1 = clk::now();
        std::vector<float> P32;
        const PinvResult pr = solve(c32.data(), K, rho, p->sigma_r, p->pinv_rtol, P32);
        const double ms_solve = ms_since(t1);
        const auto t2 = clk::now();
        const FilterPlan fp = make_plan(*p, n, rho, H, W, K);
        SavedPlanes sv{};
        if (saved != nullptr) sv = saved_at(static_cast<char*>(saved), fp);
        filter_run(c, ws, fp, f, guide, c32.data(), P32.data(), labels, out, dn, saved != nullptr ? &sv : nullptr);
        if (saved != nullptr) {
            Ctx::SavedDesc d = saved_desc(saved, saved_bytes, f, guide, n, rho, *p);
            d.K = K;
            d.H = {H};
            d.W = {W};
            d.Keff = {K};
            d.centers = c32;
            saved_register(c, std::move(d));
        }
        double ms_filter = 0.0;
        if (info) {
            FHD_HIP(hipStreamSynchronize(c.stream));
            ms_filter = ms_since(t2);
        }
        OutStats st;
        if (stats) st = out_stats(c, ws, out, N * n, dn, N);
        fill_info(info, K, pr, km.E_K, km.rounds, km.splits, ms_cluster, ms_solve, ms_filter);
        fill_stats(info, st);
        if (p->strict) strict_verdict(st);
    });
}

fhd_status fhd_filter_backward(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int H, int W,
                               const float* centers, int K, const fhd_params* p, const float* out,
                               const float* den, const float* grad_out, float* grad_f, float* grad_guide,
                               double* grad_sigma_r, double* grad_sigma_s, double* grad_centers, const void* saved,
                               size_t saved_bytes) {
    return guarded(ctx, [&](Ctx& c) {
        check_params(p, n, rho, H, W);
        FHD_REQUIRE(grad_sigma_s == nullptr || p->spatial == FHD_SPATIAL_GAUSSIAN, FHD_EUNSUPPORTED,
                    "dL/dsigma_s needs the Gaussian spatial kernel");
        FHD_REQUIRE(p->spatial != FHD_SPATIAL_YOUNG, FHD_EUNSUPPORTED,
                    "the adjoint covers the truncated Gaussian and box windows");
        FHD_REQUIRE(f && guide && centers && out && den && grad_out, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(K >= 1 && K <= 64, FHD_EUNSUPPORTED, "the adjoint supports K in [1, 64]");
        FHD_REQUIRE(p->coef == FHD_COEF_LSQ, FHD_EUNSUPPORTED, "the adjoint covers least-squares coefficients");
        const long long N = (long long)H * W;
        const size_t fb = sizeof(float) * N * n, gb = sizeof(float) * N * rho, db = sizeof(float) * N;
        auto clash = [&](const void* o, size_t ob) {
            return ranges_overlap(o, ob, f, fb) || ranges_overlap(o, ob, guide, gb) ||
                   ranges_overlap(o, ob, out, fb) || ranges_overlap(o, ob, den, db) ||
                   ranges_overlap(o, ob, grad_out, fb);
        };
        FHD_REQUIRE(!clash(grad_f, fb) && !clash(grad_guide, gb) && !ranges_overlap(grad_f, fb, grad_guide, gb),
                    FHD_EINVAL, "gradient outputs alias inputs or each other");
        FilterPlan fp = make_plan(*p, n, rho, H, W, K);
        fp.contract = FHD_CONTRACT_FP32;
        fp.materialize = true;
        Arena ws = c.arena(adjoint_workspace(fp, grad_sigma_s != nullptr, grad_centers != nullptr) + 4096);
        std::vector<float> P32;
        (void)solve(centers, K, rho, p->sigma_r, p->pinv_rtol, P32);
        std::vector<double> M((size_t)K * K);
        pinv_sigma_derivative(centers, K, rho, p->sigma_r, p->pinv_rtol, M.data());
        std::vector<float> M32(M.size());
        for (size_t q = 0; q < M.size(); ++q) M32[q] = (float)M[q];
        SavedPlanes sv{};
        if (saved != nullptr) {
            const FilterPlan ffp = saved_plan(*p, n, rho, H, W, K);
            Ctx::SavedDesc want = saved_desc(saved, saved_planes_bytes(ffp), f, guide, n, rho, *p);
            want.K = K;
            want.H = {H};
            want.W = {W};
            want.Keff = {K};
            want.centers.assign(centers, centers + (size_t)K * rho);
            saved_verify(c, want);
            FHD_REQUIRE(saved_bytes >= want.bytes, FHD_EINVAL, "saved buffer too small");
            FHD_REQUIRE(!ranges_overlap(saved, saved_bytes, grad_f, fb) &&
                            !ranges_overlap(saved, saved_bytes, grad_guide, gb),
                        FHD_EINVAL, "gradient outputs alias the saved buffer");
            sv = saved_at(static_cast<char*>(const_cast<void*>(saved)), ffp);
        }
        adjoint_run(c, ws, fp, f, guide, centers, P32.data(), M32.data(), out, den, grad_out, grad_f, grad_guide,
                    grad_sigma_r, grad_sigma_s, p->pinv_rtol, grad_centers, saved != nullptr ? &sv : nullptr);
    });
}

fhd_status fhd_filter_batch(fhd_ctx* ctx, int B, const int* H, const int* W, const long long* px_offset,
                            const float* f, int n, const float* guide, int rho, const fhd_params* p, float* out,
                            float* centers_out, int* K_eff, float* den, fhd_info* info, void* saved,
                            size_t saved_bytes) {
    return guarded(ctx, [&](Ctx& c) {
        const std::vector<long long> cnt = batch_counts(B, H, W, px_offset);
        for (int b = 0; b < B; ++b) check_params(p, n, rho, H[b], W[b]);
        reject_exact(p, "fhd_filter_batch");
        FHD_REQUIRE(f && guide && out, FHD_EINVAL, "NULL pointer");
        long long N = 0;
        for (long long q : cnt) N += q;
        FHD_REQUIRE(!ranges_overlap(out, sizeof(float) * N * n, f, sizeof(float) * N * n) &&
                        !ranges_overlap(out, sizeof(float) * N * n, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, f, sizeof(float) * N * n) &&
                        !ranges_overlap(den, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, out, sizeof(float) * N * n),
                    FHD_EINVAL, "outputs alias inputs");
        const int K = p->K;
        std::vector<size_t> soff;
        if (saved != nullptr) {
            saved_check_ptr(saved);
            saved_check_params(p, K);
            soff = saved_offsets(*p, B, H, W, n, rho);
            FHD_REQUIRE(saved_bytes >= soff[B], FHD_EINVAL, "saved buffer too small (fhd_saved_size_batch)");
            FHD_REQUIRE(!ranges_overlap(saved, saved_bytes, f, sizeof(float) * N * n) &&
                            !ranges_overlap(saved, saved_bytes, guide, sizeof(float) * N * rho) &&
                            !ranges_overlap(saved, saved_bytes, out, sizeof(float) * N * n) &&
                            !ranges_overlap(saved, saved_bytes, den, sizeof(float) * N),
                        FHD_EINVAL, "saved buffer aliases an input or output");
        }
        size_t passes = 0;
        std::vector<FilterPlan> kplans(B);  // plans at the requested K (an upper bound for K_eff)
        bool batched = true;                // one launch per pass for all images
        for (int b = 0; b < B; ++b) {
            kplans[b] = make_plan(*p, n, rho, H[b], W[b], K);
            passes = std::max(passes, filter_passes_workspace(kplans[b]));
            batched = batched && filter_batch_supported(kplans[b]);
        }
        const size_t cb = filter_consts_bytes(K, rho);
        const int ns = std::min(B, Ctx::NAUX);
        passes = align_up(passes, 256);
        const size_t fws = batched ? filter_batch_workspace(B, kplans.data()) : ns * passes;
        const size_t need = std::max(kmeans_workspace(N, rho, K, B), (size_t)B * cb + fws + 512) +
                            align_up(sizeof(int) * (size_t)N, 256) + stats_workspace(N) +
                            align_up(sizeof(StatRec) * STAT_BLOCKS * (size_t)B, 256) + 4096;
        Arena ws = c.arena(need);
        const bool hard = p->coef == FHD_COEF_HARD;
        int* labels = hard ? ws.take<int>((size_t)N) : nullptr;
        const bool stats = info != nullptr || p->strict;
        float* dn = (stats && den == nullptr) ? ws.take<float>((size_t)N) : den;
        StatRec* part = stats ? ws.take<StatRec>((size_t)STAT_BLOCKS * B) : nullptr;
        const auto t0 = clk::now();
        std::vector<KmResult> km;
        {
            Arena kws = ws;  // the clustering scratch is dead once the centers are known
            kmeans_run_batch(c, kws, guide, rho, B, px_offset, cnt.data(), K, p->kmeans_max_iter, labels, km);
        }
        const double ms_cluster = ms_since(t0);
        // all images' constants in one pinned block and one copy
        char* dev = ws.take<char>((size_t)B * cb);
        char* hs = static_cast<char*>(c.host_stage(1, (size_t)B * cb));
        std::vector<PinvResult> pr(B);
        const auto t1 = clk::now();
        parallel_for(B, [&](int b) {
            const int Kb = km[b].K_eff;
            c.last_keff = Kb;
            std::vector<float> c32((size_t)Kb * rho);
            for (size_t q = 0; q < c32.size(); ++q) c32[q] = (float)km[b].centers[q];
            if (centers_out) std::memcpy(centers_out + (size_t)b * K * rho, c32.data(), sizeof(float) * c32.size());
            if (K_eff) K_eff[b] = Kb;
            std::vector<float> P32;
            pr[b] = solve(c32.data(), Kb, rho, p->sigma_r, p->pinv_rtol, P32);
            filter_consts_fill(c32.data(), P32.data(), Kb, rho, hs + (size_t)b * cb);
        });
        const double ms_solve = ms_since(t1);
        FHD_HIP(hipMemcpyAsync(dev, hs, (size_t)B * cb, hipMemcpyHostToDevice, c.stream));
        c.stage_done(1);
        const auto t2 = clk::now();
        std::vector<SavedPlanes> sv(saved != nullptr ? B : 0);
        for (int b = 0; b < (int)sv.size(); ++b)
            sv[b] = saved_at(static_cast<char*>(saved) + soff[b], make_plan(*p, n, rho, H[b], W[b], km[b].K_eff));
        if (batched) {
            std::vector<FilterPlan> plans(B);
            std::vector<const float*> fb(B), gb(B);
            std::vector<const int*> lb(B);
            std::vector<float*> ob(B), db(B);
            std::vector<FilterConsts> kc(B);
            for (int b = 0; b < B; ++b) {
                const long long o = px_offset[b];
                plans[b] = make_plan(*p, n, rho, H[b], W[b], km[b].K_eff);
                fb[b] = f + (size_t)n * o;
                gb[b] = guide + (size_t)rho * o;
                lb[b] = hard ? labels + o : nullptr;
                ob[b] = out + (size_t)n * o;
                db[b] = dn ? dn + o : nullptr;
                kc[b] = filter_consts_at(dev + (size_t)b * cb, km[b].K_eff, rho);
            }
            filter_passes_batch(c, ws, B, plans.data(), fb.data(), gb.data(), kc.data(), hard ? lb.data() : nullptr,
                                ob.data(), dn ? db.data() : nullptr, saved != nullptr ? sv.data() : nullptr);
        } else {
            // one scratch region per stream; stream order makes it reusable image after image
            char* region = ws.take<char>((size_t)ns * passes);
            Spread sp(c, B);
            const std::vector<int> order = by_size(cnt);
            for (int i = 0; i < B; ++i) {
                const int b = order[i];
                const int k = sp.on(i);
                const FilterPlan fp = make_plan(*p, n, rho, H[b], W[b], km[b].K_eff);
                Arena pws{region + (size_t)k * passes, passes};
                const long long o = px_offset[b];
                filter_passes(c, pws, fp, f + (size_t)n * o, guide + (size_t)rho * o,
                              filter_consts_at(dev + (size_t)b * cb, km[b].K_eff, rho),
                              hard ? labels + o : nullptr, out + (size_t)n * o, dn ? dn + o : nullptr,
                              saved != nullptr ? &sv[b] : nullptr);
            }
        }
        if (saved != nullptr) {
            Ctx::SavedDesc d = saved_desc(saved, saved_bytes, f, guide, n, rho, *p);
            d.K = K;
            d.H.assign(H, H + B);
            d.W.assign(W, W + B);
            for (int b = 0; b < B; ++b) {
                d.Keff.push_back(km[b].K_eff);
                for (size_t q = 0; q < km[b].centers.size(); ++q) d.centers.push_back((float)km[b].centers[q]);
            }
            saved_register(c, std::move(d));
        }
        double ms_filter = 0.0;
        if (info) {
            FHD_HIP(hipStreamSynchronize(c.stream));
            ms_filter = ms_since(t2);
        }
        std::vector<OutStats> st(B);
        if (stats) {
            for (int b = 0; b < B; ++b)
                out_stats_launch(c, out + (size_t)n * px_offset[b], cnt[b] * n, dn + px_offset[b], cnt[b],
                                 part + (size_t)b * STAT_BLOCKS);
            std::vector<StatRec> h((size_t)STAT_BLOCKS * B);
            FHD_HIP(hipMemcpyAsync(h.data(), part, sizeof(StatRec) * h.size(), hipMemcpyDeviceToHost, c.stream));
            FHD_HIP(hipStreamSynchronize(c.stream));
            for (int b = 0; b < B; ++b) st[b] = out_stats_reduce(h.data() + (size_t)b * STAT_BLOCKS);
        }
        if (info)
            for (int b = 0; b < B; ++b) {
                fill_info(info + b, km[b].K_eff, pr[b], km[b].E_K, km[b].rounds, km[b].splits, ms_cluster, ms_solve,
                          ms_filter);
                fill_stats(info + b, st[b]);
            }
        if (p->strict)
            for (int b = 0; b < B; ++b) strict_verdict(st[b]);
    });
}

fhd_status fhd_filter_batch_backward(fhd_ctx* ctx, int B, const int* H, const int* W, const long long* px_offset,
                                     const float* f, int n, const float* guide, int rho, const float* centers,
                                     const int* K_eff, const fhd_params* p, const float* out, const float* den,
                                     const float* grad_out, float* grad_f, float* grad_guide, double* grad_sigma_r,
                                     double* grad_sigma_s, const void* saved, size_t saved_bytes) {
    return guarded(ctx, [&](Ctx& c) {
        const std::vector<long long> cnt = batch_counts(B, H, W, px_offset);
        for (int b = 0; b < B; ++b) check_params(p, n, rho, H[b], W[b]);
        FHD_REQUIRE(grad_sigma_s == nullptr || p->spatial == FHD_SPATIAL_GAUSSIAN, FHD_EUNSUPPORTED,
                    "dL/dsigma_s needs the Gaussian spatial kernel");
        FHD_REQUIRE(p->spatial != FHD_SPATIAL_YOUNG, FHD_EUNSUPPORTED,
                    "the adjoint covers the truncated Gaussian and box windows");
        const bool with_s = grad_sigma_s != nullptr;
        FHD_REQUIRE(f && guide && centers && K_eff && out && den && grad_out, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(p->coef == FHD_COEF_LSQ, FHD_EUNSUPPORTED, "the adjoint covers least-squares coefficients");
        const int K = p->K;
        long long N = 0;
        for (long long q : cnt) N += q;
        const size_t fb = sizeof(float) * N * n, gb = sizeof(float) * N * rho, db = sizeof(float) * N;
        auto clash = [&](const void* o, size_t ob) {
            return ranges_overlap(o, ob, f, fb) || ranges_overlap(o, ob, guide, gb) ||
                   ranges_overlap(o, ob, out, fb) || ranges_overlap(o, ob, den, db) ||
                   ranges_overlap(o, ob, grad_out, fb);
        };
        FHD_REQUIRE(!clash(grad_f, fb) && !clash(grad_guide, gb) && !ranges_overlap(grad_f, fb, grad_guide, gb),
                    FHD_EINVAL, "gradient outputs alias inputs or each other");
        std::vector<FilterPlan> plans(B);
        size_t passes = 0;
        bool batched = !with_s;  // dL/dsigma_s: the per-image adjoints
        for (int b = 0; b < B; ++b) {
            FHD_REQUIRE(K_eff[b] >= 1 && K_eff[b] <= std::min(K, 64), FHD_EUNSUPPORTED,
                        "the adjoint supports K_eff in [1, min(K, 64)]");
            plans[b] = make_plan(*p, n, rho, H[b], W[b], K_eff[b]);
            plans[b].contract = FHD_CONTRACT_FP32;
            plans[b].materialize = true;
            passes = std::max(passes, adjoint_passes_workspace(plans[b], with_s, false));
            batched = batched && adjoint_batch_supported(plans[b]);
        }
        std::vector<SavedPlanes> sv;
        if (saved != nullptr) {
            const std::vector<size_t> soff = saved_offsets(*p, B, H, W, n, rho);
            Ctx::SavedDesc want = saved_desc(saved, soff[B], f, guide, n, rho, *p);
            want.K = K;
            want.H.assign(H, H + B);
            want.W.assign(W, W + B);
            want.Keff.assign(K_eff, K_eff + B);
            for (int b = 0; b < B; ++b)
                want.centers.insert(want.centers.end(), centers + (size_t)b * K * rho,
                                    centers + (size_t)b * K * rho + (size_t)K_eff[b] * rho);
            saved_verify(c, want);
            FHD_REQUIRE(saved_bytes >= soff[B], FHD_EINVAL, "saved buffer too small");
            FHD_REQUIRE(!ranges_overlap(saved, saved_bytes, grad_f, fb) &&
                            !ranges_overlap(saved, saved_bytes, grad_guide, gb),
                        FHD_EINVAL, "gradient outputs alias the saved buffer");
            for (int b = 0; b < B; ++b)
                sv.push_back(saved_at(static_cast<char*>(const_cast<void*>(saved)) + soff[b],
                                      saved_plan(*p, n, rho, H[b], W[b], K_eff[b])));
        }
        const size_t cb = adjoint_consts_bytes(K, rho);
        const int ns = std::min(B, Ctx::NAUX);
        passes = align_up(passes, 256);
        const size_t region = batched ? adjoint_batch_workspace(B, plans.data()) : ns * passes;
        Arena ws = c.arena((size_t)B * cb + 2 * align_up(sizeof(double) * (B + 1), 256) + region + 4096);
        char* dev = ws.take<char>((size_t)B * cb);
        double* sig = ws.take<double>((size_t)B + 1);
        double* sigs = ws.take<double>((size_t)B + 1);
        char* hs = static_cast<char*>(c.host_stage(1, (size_t)B * cb));
        parallel_for(B, [&](int b) {
            const int Kb = K_eff[b];
            const float* cen = centers + (size_t)b * K * rho;
            std::vector<float> P32;
            (void)solve(cen, Kb, rho, p->sigma_r, p->pinv_rtol, P32);
            std::vector<double> M((size_t)Kb * Kb);
            pinv_sigma_derivative(cen, Kb, rho, p->sigma_r, p->pinv_rtol, M.data());
            char* h = hs + (size_t)b * cb;
            filter_consts_fill(cen, P32.data(), Kb, rho, h);
            float* m32 = reinterpret_cast<float*>(h + filter_consts_bytes(Kb, rho));
            for (size_t q = 0; q < M.size(); ++q) m32[q] = (float)M[q];
        });
        FHD_HIP(hipMemcpyAsync(dev, hs, (size_t)B * cb, hipMemcpyHostToDevice, c.stream));
        c.stage_done(1);
        if (batched) {
            std::vector<const float*> fb_(B), gb_(B), Mb(B), ob(B), db_(B), gob(B);
            std::vector<float*> gfb(B), ggb(B);
            std::vector<FilterConsts> kc(B);
            for (int b = 0; b < B; ++b) {
                const int Kb = K_eff[b];
                const long long o = px_offset[b];
                const char* d = dev + (size_t)b * cb;
                kc[b] = filter_consts_at(d, Kb, rho);
                Mb[b] = reinterpret_cast<const float*>(d + filter_consts_bytes(Kb, rho));
                fb_[b] = f + (size_t)n * o;
                gb_[b] = guide + (size_t)rho * o;
                ob[b] = out + (size_t)n * o;
                db_[b] = den + o;
                gob[b] = grad_out + (size_t)n * o;
                gfb[b] = grad_f ? grad_f + (size_t)n * o : nullptr;
                ggb[b] = grad_guide ? grad_guide + (size_t)rho * o : nullptr;
            }
            adjoint_passes_batch(c, ws, B, plans.data(), fb_.data(), gb_.data(), kc.data(), Mb.data(), ob.data(),
                                 db_.data(), gob.data(), gfb.data(), ggb.data(), sig + B,
                                 saved != nullptr ? sv.data() : nullptr);
        } else {
            char* region = ws.take<char>((size_t)ns * passes);
            Spread sp(c, B);
            const std::vector<int> order = by_size(cnt);
            for (int i = 0; i < B; ++i) {
                const int b = order[i];
                const int k = sp.on(i);
                const int Kb = K_eff[b];
                const long long o = px_offset[b];
                const char* d = dev + (size_t)b * cb;
                Arena pws{region + (size_t)k * passes, passes};
                adjoint_passes(c, pws, plans[b], f + (size_t)n * o, guide + (size_t)rho * o,
                               filter_consts_at(d, Kb, rho),
                               reinterpret_cast<const float*>(d + filter_consts_bytes(Kb, rho)), out + (size_t)n * o,
                               den + o, grad_out + (size_t)n * o, grad_f ? grad_f + (size_t)n * o : nullptr,
                               grad_guide ? grad_guide + (size_t)rho * o : nullptr, sig + b,
                               with_s ? sigs + b : nullptr, nullptr, saved != nullptr ? &sv[b] : nullptr);
            }
        }
        if (grad_sigma_r != nullptr) {
            if (!batched) sum_doubles(c, sig, B, sig + B);
            FHD_HIP(hipMemcpyAsync(grad_sigma_r, sig + B, sizeof(double), hipMemcpyDeviceToHost, c.stream));
        }
        if (with_s) {
            sum_doubles(c, sigs, B, sigs + B);
            FHD_HIP(hipMemcpyAsync(grad_sigma_s, sigs + B, sizeof(double), hipMemcpyDeviceToHost, c.stream));
        }
        if (grad_sigma_r != nullptr || with_s) FHD_HIP(hipStreamSynchronize(c.stream));
    });
}

fhd_status fhd_bruteforce(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int H, int W,
                          const fhd_params* p, float* out, float* den) {
    return guarded(ctx, [&](Ctx& c) {
        check_params(p, n, rho, H, W);
        FHD_REQUIRE(p->spatial != FHD_SPATIAL_YOUNG, FHD_EUNSUPPORTED,
                    "the brute force evaluates eqs. (1)-(2) with a finite window");
        FHD_REQUIRE(f && guide && out, FHD_EINVAL, "NULL pointer");
        const long long N = (long long)H * W;
        FHD_REQUIRE(!ranges_overlap(out, sizeof(float) * N * n, f, sizeof(float) * N * n) &&
                        !ranges_overlap(out, sizeof(float) * N * n, guide, sizeof(float) * N * rho),
                    FHD_EINVAL, "outputs alias inputs");
        const FilterPlan fp = make_plan(*p, n, rho, H, W, 1);
        bruteforce_run(c, fp, f, guide, out, den);
        if (p->strict) {
            Arena ws = c.arena(stats_workspace(0) + 4096);
            strict_verdict(out_stats(c, ws, out, N * n, den, N));
        }
    });
}

fhd_status fhd_nlm_guide(fhd_ctx* ctx, const float* f, int n, int H, int W, int patch, int dims, float* guide,
                         double* eigvals) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(f != nullptr && guide != nullptr, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(n >= 1 && H >= 1 && W >= 1 && patch >= 1, FHD_EINVAL, "n, H, W, patch must be >= 1");
        FHD_REQUIRE((long long)H * W < (1LL << 31), FHD_EUNSUPPORTED, "image has 2^31 pixels or more");
        const long long N = (long long)H * W;
        FHD_REQUIRE(!ranges_overlap(guide, sizeof(float) * N * dims, f, sizeof(float) * N * n), FHD_EINVAL,
                    "guide aliases the image");
        Arena ws = c.arena(nlm_workspace(n, H, W, patch, dims));
        nlm_guide_run(c, ws, f, n, H, W, patch, dims, guide, eigvals);
        if (eigvals) FHD_HIP(hipStreamSynchronize(c.stream));
    });
}

fhd_status fhd_filter_volume(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int D, int H, int W,
                             const fhd_params* p, float* out, float* centers_out, float* den, fhd_info* info) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(D >= 1 && H >= 1, FHD_EINVAL, "D and H must be >= 1");
        FHD_REQUIRE((long long)D * H <= 65535, FHD_EUNSUPPORTED, "a volume takes at most 65535 rows (D * H)");
        check_params(p, n, rho, D * H, W);
        FHD_REQUIRE(p->spatial != FHD_SPATIAL_YOUNG, FHD_EUNSUPPORTED,
                    "volumes take the Gaussian or box window (finite, separable over [-S,S]^3)");
        FHD_REQUIRE(p->contract == FHD_CONTRACT_FP32, FHD_EUNSUPPORTED, "volumes take the FP32 form");
        reject_exact(p, "fhd_filter_volume");
        FHD_REQUIRE(f && guide && out, FHD_EINVAL, "NULL pointer");
        const long long N = (long long)D * H * W;
        FHD_REQUIRE(!ranges_overlap(out, sizeof(float) * N * n, f, sizeof(float) * N * n) &&
                        !ranges_overlap(out, sizeof(float) * N * n, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, f, sizeof(float) * N * n) &&
                        !ranges_overlap(den, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, out, sizeof(float) * N * n),
                    FHD_EINVAL, "outputs alias inputs");
        FHD_REQUIRE((long long)p->K * (n + 1) * N / 256 < (1LL << 31), FHD_EUNSUPPORTED,
                    "too many plane voxels for one launch");
        size_t need = 0;
        {
            const FilterPlan fp0 = make_plan(*p, n, rho, D * H, W, p->K);
            need = kmeans_workspace(N, rho, p->K) + filter_volume_workspace(fp0) +
                   align_up(sizeof(int) * (size_t)N, 256) + stats_workspace(N) + 4096;
        }
        Arena ws = c.arena(need);
        const bool hard = p->coef == FHD_COEF_HARD;
        int* labels = hard ? ws.take<int>((size_t)N) : nullptr;
        const bool stats = info != nullptr || p->strict;
        float* dn = (stats && den == nullptr) ? ws.take<float>((size_t)N) : den;
        const auto t0 = clk::now();
        KmResult km;
        {
            Arena kws = ws;  // the clustering scratch is dead once the centers are known
            kmeans_run(c, kws, guide, rho, N, p->K, p->kmeans_max_iter, labels, km);
        }
        const double ms_cluster = ms_since(t0);
        const int K = km.K_eff;
        c.last_keff = K;
        std::vector<float> c32((size_t)K * rho);
        for (size_t q = 0; q < c32.size(); ++q) c32[q] = (float)km.centers[q];
        if (centers_out) std::memcpy(centers_out, c32.data(), sizeof(float) * c32.size());
        const auto t1 = clk::now();
        std::vector<float> P32;
        const PinvResult pr = solve(c32.data(), K, rho, p->sigma_r, p->pinv_rtol, P32);
        const double ms_solve = ms_since(t1);
        const auto t2 = clk::now();
        const FilterPlan fp = make_plan(*p, n, rho, D * H, W, K);
        filter_volume_run(c, ws, fp, D, f, guide, c32.data(), P32.data(), labels, out, dn);
        double ms_filter = 0.0;
        if (info) {
            FHD_HIP(hipStreamSynchronize(c.stream));
            ms_filter = ms_since(t2);
        }
        OutStats st;
        if (stats) st = out_stats(c, ws, out, N * n, dn, N);
        fill_info(info, K, pr, km.E_K, km.rounds, km.splits, ms_cluster, ms_solve, ms_filter);
        fill_stats(info, st);
        if (p->strict) strict_verdict(st);
    });
}

fhd_status fhd_bruteforce_volume(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int D, int H,
                                 int W, const fhd_params* p, float* out, float* den) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(D >= 1 && H >= 1, FHD_EINVAL, "D and H must be >= 1");
        FHD_REQUIRE((long long)D * H <= 65535, FHD_EUNSUPPORTED, "a volume takes at most 65535 rows (D * H)");
        check_params(p, n, rho, D * H, W);
        FHD_REQUIRE(p->spatial != FHD_SPATIAL_YOUNG, FHD_EUNSUPPORTED,
                    "the brute force evaluates eqs. (1)-(2) with a finite window");
        FHD_REQUIRE(f && guide && out, FHD_EINVAL, "NULL pointer");
        const long long N = (long long)D * H * W;
        FHD_REQUIRE(!ranges_overlap(out, sizeof(float) * N * n, f, sizeof(float) * N * n) &&
                        !ranges_overlap(out, sizeof(float) * N * n, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, f, sizeof(float) * N * n) &&
                        !ranges_overlap(den, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(den, sizeof(float) * N, out, sizeof(float) * N * n),
                    FHD_EINVAL, "outputs alias inputs");
        const FilterPlan fp = make_plan(*p, n, rho, D * H, W, 1);
        bruteforce_volume_run(c, fp, D, f, guide, out, den);
        if (p->strict) {
            Arena ws = c.arena(stats_workspace(0) + 4096);
            strict_verdict(out_stats(c, ws, out, N * n, den, N));
        }
    });
}

fhd_status fhd_approx_error(fhd_ctx* ctx, const float* guide, int rho, int H, int W, const float* centers, int K,
                            const fhd_params* p, float* err, double* mean) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(p != nullptr, FHD_EINVAL, "params is NULL");
        FHD_REQUIRE(guide != nullptr && centers != nullptr, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(err != nullptr || mean != nullptr, FHD_EINVAL, "neither err nor mean requested");
        FHD_REQUIRE(rho >= 1 && H >= 1 && W >= 1, FHD_EINVAL, "rho, H, W must be >= 1");
        FHD_REQUIRE(rho <= FHD_MAX_RHO, FHD_EUNSUPPORTED, "rho exceeds FHD_MAX_RHO");
        FHD_REQUIRE((long long)H * W < (1LL << 31), FHD_EUNSUPPORTED, "image has 2^31 pixels or more");
        FHD_REQUIRE(K >= 1, FHD_EINVAL, "K must be >= 1");
        FHD_REQUIRE(K <= 64, FHD_EUNSUPPORTED, "the approximation error takes at most 64 clusters");
        FHD_REQUIRE(p->sigma_r > 0.0f && !std::isnan(p->sigma_r), FHD_EINVAL, "sigma_r must be > 0");
        FHD_REQUIRE(p->spatial == FHD_SPATIAL_GAUSSIAN || p->spatial == FHD_SPATIAL_BOX, FHD_EINVAL,
                    "the window of eq. (10) needs the Gaussian (radius from sigma_s) or box spatial kernel");
        if (p->spatial == FHD_SPATIAL_GAUSSIAN && p->radius < 0)
            FHD_REQUIRE(p->sigma_s > 0.0f && std::isfinite(p->sigma_s), FHD_EINVAL, "sigma_s must be > 0");
        if (p->spatial == FHD_SPATIAL_BOX) FHD_REQUIRE(p->radius >= 0, FHD_EINVAL, "the box kernel needs radius >= 0");
        const int S = resolve_radius(*p);
        FHD_REQUIRE(S >= 0 && S <= FHD_MAX_RADIUS, FHD_EUNSUPPORTED, "radius exceeds FHD_MAX_RADIUS");
        const long long N = (long long)H * W;
        FHD_REQUIRE(!ranges_overlap(err, sizeof(float) * N, guide, sizeof(float) * N * rho), FHD_EINVAL,
                    "err aliases the guide");
        std::vector<float> P32;
        solve(centers, K, rho, p->sigma_r, p->pinv_rtol, P32);
        Arena ws = c.arena(approx_error_workspace(H, W, K, rho));
        approx_error_run(c, ws, guide, rho, H, W, centers, P32.data(), K, S, p->sigma_r, err, mean);
    });
}

fhd_status fhd_exact_ls(fhd_ctx* ctx, const float* guide, int rho, int H, int W, const float* centers, int K,
                        const fhd_params* p, float* coef, float* obj, float* obj11) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(p != nullptr, FHD_EINVAL, "params is NULL");
        FHD_REQUIRE(guide != nullptr && centers != nullptr, FHD_EINVAL, "NULL pointer");
        FHD_REQUIRE(coef != nullptr || obj != nullptr || obj11 != nullptr, FHD_EINVAL, "no output requested");
        FHD_REQUIRE(rho >= 1 && H >= 1 && W >= 1, FHD_EINVAL, "rho, H, W must be >= 1");
        FHD_REQUIRE(rho <= FHD_MAX_RHO, FHD_EUNSUPPORTED, "rho exceeds FHD_MAX_RHO");
        FHD_REQUIRE((long long)H * W < (1LL << 31), FHD_EUNSUPPORTED, "image has 2^31 pixels or more");
        FHD_REQUIRE(K >= 1, FHD_EINVAL, "K must be >= 1");
        FHD_REQUIRE(K <= EXACT_LS_MAX_K, FHD_EUNSUPPORTED, "the per-pixel least squares takes at most 32 clusters");
        FHD_REQUIRE(p->sigma_r > 0.0f && !std::isnan(p->sigma_r), FHD_EINVAL, "sigma_r must be > 0");
        FHD_REQUIRE(p->spatial == FHD_SPATIAL_GAUSSIAN || p->spatial == FHD_SPATIAL_BOX, FHD_EINVAL,
                    "the window of eq. (10) needs the Gaussian (radius from sigma_s) or box spatial kernel");
        if (p->spatial == FHD_SPATIAL_GAUSSIAN && p->radius < 0)
            FHD_REQUIRE(p->sigma_s > 0.0f && std::isfinite(p->sigma_s), FHD_EINVAL, "sigma_s must be > 0");
        if (p->spatial == FHD_SPATIAL_BOX) FHD_REQUIRE(p->radius >= 0, FHD_EINVAL, "the box kernel needs radius >= 0");
        const int S = resolve_radius(*p);
        FHD_REQUIRE(S >= 0 && S <= FHD_MAX_RADIUS, FHD_EUNSUPPORTED, "radius exceeds FHD_MAX_RADIUS");
        const long long N = (long long)H * W;
        FHD_REQUIRE(!ranges_overlap(coef, sizeof(float) * N * K, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(obj, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(obj11, sizeof(float) * N, guide, sizeof(float) * N * rho) &&
                        !ranges_overlap(obj, sizeof(float) * N, coef, sizeof(float) * N * K) &&
                        !ranges_overlap(obj11, sizeof(float) * N, coef, sizeof(float) * N * K) &&
                        !ranges_overlap(obj, sizeof(float) * N, obj11, sizeof(float) * N),
                    FHD_EINVAL, "outputs alias an input or each other");
        // A^+ in FP64 (eq. (10) at the surrogate's coefficients), the centers
        std::vector<double> A((size_t)K * K), P((size_t)K * K);
        kernel_matrix(centers, K, rho, p->sigma_r, A.data());
        pinv_symmetric(A.data(), K, p->pinv_rtol, P.data());
        const size_t mb = align_up(sizeof(float) * K * rho, 256), pb = sizeof(double) * K * K;
        Arena ws = c.arena(mb + pb + 512);
        char* dev = ws.take<char>(mb + pb);
        char* hs = static_cast<char*>(c.host_stage(1, mb + pb));
        std::memcpy(hs, centers, sizeof(float) * K * rho);
        std::memcpy(hs + mb, P.data(), pb);
        FHD_HIP(hipMemcpyAsync(dev, hs, mb + pb, hipMemcpyHostToDevice, c.stream));
        c.stage_done(1);
        exact_ls_run(c, guide, rho, H, W, reinterpret_cast<const float*>(dev), K,
                     reinterpret_cast<const double*>(dev + mb), p->sigma_r, S, coef, N, W, obj, obj11);
    });
}

int fhd_last_k_eff(const fhd_ctx* ctx) { return ctx == nullptr ? 0 : ctx->impl.last_keff; }

fhd_status fhd_scale_guide(fhd_ctx* ctx, const float* guide, int rho, long long N, const float* sigma_d,
                           float* out) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(sigma_d != nullptr, FHD_EINVAL, "sigma_d is NULL");
        FHD_REQUIRE(rho >= 1 && rho <= FHD_MAX_RHO, FHD_EINVAL, "rho must be in [1, FHD_MAX_RHO]");
        FHD_REQUIRE(N >= 0, FHD_EINVAL, "N must be >= 0");
        FHD_REQUIRE(N < (1LL << 38) / rho, FHD_EUNSUPPORTED, "guide has 2^38 entries or more");
        RangeScales sc{};
        for (int d = 0; d < rho; ++d) {
            FHD_REQUIRE(std::isfinite(sigma_d[d]) && sigma_d[d] > 0.0f, FHD_EINVAL,
                        "every sigma_d must be finite and > 0");
            sc.s[d] = sigma_d[d];
        }
        if (N == 0) return;
        FHD_REQUIRE(guide != nullptr && out != nullptr, FHD_EINVAL, "NULL pointer");
        const size_t bytes = sizeof(float) * (size_t)N * rho;
        FHD_REQUIRE(out == guide || !ranges_overlap(out, bytes, guide, bytes), FHD_EINVAL,
                    "out overlaps guide without being equal to it");
        const long long blocks = (N * rho + 255) / 256;
        hipLaunchKernelGGL(scale_guide_kernel, dim3((unsigned)blocks), dim3(256), 0, c.stream, guide, N, rho, sc,
                           out);
        FHD_HIP(hipGetLastError());
    });
}

fhd_status fhd_timing_enable(fhd_ctx* ctx, int enable) {
    return guarded(ctx, [&](Ctx& c) { c.timing = enable != 0; });
}

fhd_status fhd_timing_units(fhd_ctx* ctx, long long* units) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(units != nullptr, FHD_EINVAL, "NULL pointer");
        for (int s = 0; s < FHD_NUM_STAGES; ++s) {
            units[s] = c.units[s];
            c.units[s] = 0;
        }
    });
}

fhd_status fhd_timing_read(fhd_ctx* ctx, double* ms, int* launches) {
    return guarded(ctx, [&](Ctx& c) {
        FHD_REQUIRE(ms != nullptr && launches != nullptr, FHD_EINVAL, "NULL pointer");
        FHD_HIP(hipStreamSynchronize(c.stream));
        for (int s = 0; s < FHD_NUM_STAGES; ++s) {
            double tot = 0.0;
            int nl = 0;
            for (auto& pr : c.ev_rec[s]) {
                float t = 0.0f;
                FHD_HIP(hipEventElapsedTime(&t, pr.begin, pr.end));
                tot += t;
                nl += pr.launches;
                c.ev_pool.push_back(pr.begin);
                c.ev_pool.push_back(pr.end);
            }
            ms[s] = tot;
            launches[s] = nl;
            c.ev_rec[s].clear();
        }
    });
}

}  // extern "C"
