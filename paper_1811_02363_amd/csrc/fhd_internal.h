// Internal declarations shared by the HIP sources of libfhd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fhd.h"

namespace fhd {

// A failure inside the library; converted to a status code at the C ABI.
struct Error : std::runtime_error {
    fhd_status status;
    Error(fhd_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define FHD_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::fhd::Error(FHD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define FHD_REQUIRE(cond, status, msg)                         \
    do {                                                       \
        if (!(cond)) throw ::fhd::Error((status), (msg));      \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over one device buffer.  Every slice is 256-byte aligned.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    template <class T>
    T* take(size_t count) {
        size_t off = align_up(used, 256);
        size_t bytes = align_up(count * sizeof(T), 256);
        if (base != nullptr && off + bytes > cap)
            throw Error(FHD_ENOMEM, "workspace too small");
        used = off + bytes;
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
};

struct Ctx;

// ---- clustering (kmeans.hip) ------------------------------------------------
struct KmResult {
    int K_eff = 0;
    int rounds = 0;
    int splits = 0;
    double E_K = 0.0;
    std::vector<double> centers;   // K_eff x rho, FP64 leaf centroids in heap order
};
// Workspace bytes for clustering N points of dimension rho into <= K leaves.
size_t kmeans_workspace(long long N, int rho, int K, int images = 1);
void kmeans_run(Ctx& c, Arena& ws, const float* guide, int rho, long long N, int K,
                int max_iter, int* labels, KmResult& out);
// Several images (planar rho x N_b guides at element offsets rho * px_offset[b],
// packed back to back), one tree each, every pass launched once for all trees.
// labels (optional) index the concatenation of the images.
void kmeans_run_batch(Ctx& c, Arena& ws, const float* guide, int rho, int images,
                      const long long* px_offset, const long long* px_count, int K, int max_iter,
                      int* labels, std::vector<KmResult>& out);

// ---- K x K solve (linalg.cpp) ----------------------------------------------
struct PinvResult {
    int rank = 0;
    double cond = 0.0;
    double max_abs = 0.0;
};
// A (K x K, row-major) = phi(mu_k - mu_l) from FP32 centers promoted to FP64.
void kernel_matrix(const float* centers, int K, int rho, double sigma_r, double* A);
// Pseudo-inverse of the symmetric A; rtol <= 0: K * 2^-52 relative to s_max.
PinvResult pinv_symmetric(const double* A, int K, double rtol, double* P);
void pinv_sigma_derivative(const float* centers, int K, int rho, double sigma_r, double rtol, double* M);
// dL/dmu (K x rho) from the adjoint's pixel sums: Gm = sum_i gamma(i) b(i)^T
// (K x K, = dL/dA^+), S1_l = sum_i w_l(i), S2_l = sum_i w_l(i) p(i) (K x rho),
// w_l = dL/db_l b_l; the pseudo-inverse's rank held fixed.
void centers_gradient(const float* centers, int K, int rho, double sigma_r, double rtol, const double* Gm,
                      const double* S1, const double* S2, double* grad);
// Symmetric eigen-decomposition (t destroyed): eigenvalues lam (unsorted),
// column i of v (row-major n x n) the i-th unit eigenvector.  false: the QR
// iteration did not converge (or produced non-finite eigenvalues).
bool sym_eigen(std::vector<double>& t, int n, std::vector<double>& lam, std::vector<double>& v);
// sym_eigen, failing with FHD_ENUMERIC ("eigen-decomposition of <what> ...")
// when it does not converge.
void sym_eigen_checked(std::vector<double>& t, int n, std::vector<double>& lam, std::vector<double>& v,
                       const char* what);

// ---- filter passes (filter.hip) --------------------------------------------
struct FilterPlan {
    int n, rho, H, W, K, S, spatial, contract, coef;
    float sigma_s, sigma_r;
    long long N;
    int Wp;                // row pitch of the intermediate planes (floats)
    bool materialize;      // B and C planes are computed by a separate pass
};
size_t filter_workspace(const FilterPlan& fp);
// The forward's intermediates kept for the adjoint in a caller buffer: the
// row-filtered planes (the layout of the intermediate planes), the C planes
// and, when the weights are materialised, the B planes (each K x H x Wp).
struct SavedPlanes {
    float* planes;
    float* C;
    float* B;
};
size_t saved_planes_bytes(const FilterPlan& fp);
SavedPlanes saved_at(char* base, const FilterPlan& fp);
void filter_run(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                const float* centers_host, const float* Pfp32_host, const int* labels,
                float* out, float* den, const SavedPlanes* sv = nullptr);
// Device copies of one image's constants: centers (K x rho), A^+ (K x K) and
// the contraction offset (rho), FP32, in one block of filter_consts_bytes.
// Eq. (10) per pixel (exact_ls.hip): c*(i) into `coef` (K planes, plane
// stride cstride, row pitch cpitch) and the objective at c* (obj) and at
// A^+ b(i) (obj11, needs P_dev: K x K FP64); any output may be null.
constexpr int EXACT_LS_MAX_K = 32;
void exact_ls_run(Ctx& c, const float* guide, int rho, int H, int W, const float* mu_dev, int K,
                  const double* P_dev, double sigma_r, int S, float* coef, long long cstride, int cpitch, float* obj,
                  float* obj11);

struct FilterConsts {
    const float* mu;
    const float* P;
    const float* offs;
};
size_t filter_consts_bytes(int K, int rho);
void filter_consts_fill(const float* centers, const float* P32, int K, int rho, char* host_dst);
FilterConsts filter_consts_at(const char* dev, int K, int rho);
size_t filter_passes_workspace(const FilterPlan& fp);
// One launch per pass for all images of a batch (weights inline, radius 1..32).
bool filter_batch_supported(const FilterPlan& fp);
size_t filter_batch_workspace(int B, const FilterPlan* plans);
void filter_passes_batch(Ctx& c, Arena& ws, int B, const FilterPlan* plans, const float* const* f,
                         const float* const* guide, const FilterConsts* kc, const int* const* labels,
                         float* const* out, float* const* den, const SavedPlanes* sv = nullptr);
void filter_passes(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                   const FilterConsts& kc, const int* labels, float* out, float* den,
                   const SavedPlanes* sv = nullptr);
void bruteforce_run(Ctx& c, const FilterPlan& fp, const float* f, const float* guide,
                    float* out, float* den);
// with_s: also the dL/dsigma_s passes (one more K-plane set)
// with_mu: also the pixel sums of the centers gradient
size_t adjoint_workspace(const FilterPlan& fp, bool with_s, bool with_mu);
// constants of the adjoint: filter constants, then M = dA^+/dsigma_r (K x K)
size_t adjoint_consts_bytes(int K, int rho);
size_t adjoint_passes_workspace(const FilterPlan& fp, bool with_s, bool with_mu);
// writes the sigma_r gradient (one double) to sig_dev on the device, and the
// sigma_s gradient to sigs_dev when it is not null (Gaussian kernel only),
// and the centers gradient's pixel sums [Gm (K x K), S1 (K), S2 (K x rho)]
// to mu_dev when it is not null
void adjoint_passes(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                    const FilterConsts& kc, const float* Md, const float* out, const float* den,
                    const float* gout, float* gradf, float* gradp, double* sig_dev, double* sigs_dev,
                    double* mu_dev, const SavedPlanes* sv = nullptr);
// One launch per pass for the adjoint of all images of a batch (guides of at
// most 8 dimensions, at most 32 clusters, radius 1..32); per-image pointers;
// the sigma_r gradient summed over all images goes to sig_dev.
bool adjoint_batch_supported(const FilterPlan& fp);
size_t adjoint_batch_workspace(int B, const FilterPlan* plans);
void adjoint_passes_batch(Ctx& c, Arena& ws, int B, const FilterPlan* plans, const float* const* f,
                          const float* const* guide, const FilterConsts* kc, const float* const* Md,
                          const float* const* out, const float* const* den, const float* const* gout,
                          float* const* gradf, float* const* gradp, double* sig_dev,
                          const SavedPlanes* sv = nullptr);
// out_dev[0] = v[0] + ... + v[count-1] (fixed order), on the ctx stream
void sum_doubles(Ctx& c, const double* v, int count, double* out_dev);
void adjoint_run(Ctx& c, Arena& ws, const FilterPlan& fp, const float* f, const float* guide,
                 const float* centers_host, const float* Pfp32_host, const float* M_host, const float* out,
                 const float* den, const float* gout, float* gradf, float* gradp, double* gsig,
                 double* gsigs, double rtol, double* gmu, const SavedPlanes* sv = nullptr);

// A 3-D domain: the plan's H is D slices of H / D rows; FP32 weights
// materialised, three 1-D passes over [-S,S]^3, then the recombination
// (S = fp.S, no halo rows); labels (per voxel) for the hard variant.
size_t filter_volume_workspace(const FilterPlan& fp);
void filter_volume_run(Ctx& c, Arena& ws, const FilterPlan& fp, int D, const float* f, const float* guide,
                       const float* centers_host, const float* Pfp32_host, const int* labels, float* out,
                       float* den);
void bruteforce_volume_run(Ctx& c, const FilterPlan& fp, int D, const float* f, const float* guide, float* out,
                           float* den);
// Error of the kernel approximation (eq. (10) at c = A^+ b) per pixel (err,
// may be null) and its pixel mean (mean, may be null; synchronises); K <= 64.
size_t approx_error_workspace(int H, int W, int K, int rho);
void approx_error_run(Ctx& c, Arena& ws, const float* guide, int rho, int H, int W, const float* centers_host,
                      const float* Pfp32_host, int K, int S, float sigma_r, float* err, double* mean);

// ---- nonlocal-means guide (nlm.hip) ----------------------------------------
size_t nlm_workspace(int n, int H, int W, int m, int dims);
void nlm_guide_run(Ctx& c, Arena& ws, const float* f, int n, int H, int W, int m, int dims, float* guide,
                   double* eigvals);

// ---- context ---------------------------------------------------------------
struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // library-owned workspace
    void* own_ws = nullptr;
    size_t own_bytes = 0;
    // caller-owned workspace
    void* ext_ws = nullptr;
    size_t ext_bytes = 0;
    // pinned host staging slots (0: clustering, 1: filter uploads, 2: misc);
    // each slot's event marks the end of the last copy that read it
    void* pinned[3] = {nullptr, nullptr, nullptr};
    size_t pinned_bytes[3] = {0, 0, 0};
    hipEvent_t pinned_ev[3] = {nullptr, nullptr, nullptr};
    bool pinned_pending[3] = {false, false, false};
    // orders a new stream (fhd_set_stream) after the work on the previous one
    hipEvent_t switch_ev = nullptr;
    // what the recent forward calls wrote into caller buffers for their
    // adjoints (most recent last): the adjoint accepts a saved buffer only
    // with the arguments of the forward call that wrote it
    struct SavedDesc {
        const void* ptr = nullptr;
        size_t bytes = 0;
        const float* f = nullptr;
        const float* guide = nullptr;
        int n = 0, rho = 0, K = 0, S = 0, spatial = 0;
        float sigma_s = 0.0f, sigma_r = 0.0f;
        double rtol = 0.0;
        std::vector<int> H, W, Keff;     // per image (one for the single-image calls)
        std::vector<float> centers;      // the K_eff rows of every image
    };
    std::vector<SavedDesc> saved;
    // allocation-free entry point: the device address of this GPU's static
    // scratch array, and a pinned buffer for the constants (made by
    // fhd_create, sized for FHD_MAX_K and FHD_MAX_RHO) with the event that
    // marks the end of the last copy out of it
    char* noalloc_scratch = nullptr;
    void* noalloc_pinned = nullptr;
    hipEvent_t noalloc_ev = nullptr;
    bool noalloc_pending = false;

    // stage timing (fhd_timing_enable)
    bool timing = false;
    int last_keff = 0;  // K_eff of the last call that clustered
    std::vector<hipEvent_t> ev_pool;
    struct EvPair {
        hipEvent_t begin, end;
        int launches;  // kernel launches between the two events
    };
    std::vector<EvPair> ev_rec[FHD_NUM_STAGES];
    long long units[FHD_NUM_STAGES] = {};  // algorithmic work per stage (fhd_timing_units)
    hipEvent_t take_event();
    // Records the start of `stage` now; returns the event (null when off).
    hipEvent_t stage_begin();
    void stage_end(int stage, hipEvent_t begin, int launches = 1);

    // auxiliary streams (default priority) for the independent per-image
    // work of a batch: fork(n) makes aux[0..n) wait for what `stream` has
    // enqueued so far, join(n) makes `stream` wait for aux[0..n)
    static constexpr int NAUX = 4;
    hipStream_t aux[NAUX] = {};
    hipEvent_t aux_ev[NAUX + 1] = {};
    void fork(int n);
    void join(int n);

    Arena arena(size_t need);
    // A pinned buffer of at least `bytes`, safe to overwrite (waits for the
    // copies enqueued from it before the last stage_done(slot)).
    void* host_stage(int slot, size_t bytes);
    void stage_done(int slot);
    void release();
};

}  // namespace fhd

struct fhd_ctx {
    fhd::Ctx impl;
};
