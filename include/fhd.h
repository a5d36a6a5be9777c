/*
 * fhd.h - C ABI of the MI355X (gfx950) fast high-dimensional bilateral and
 * nonlocal-means filter of Nair & Chaudhury, "Fast High-Dimensional Bilateral
 * and Nonlocal Means Filtering" (IEEE TIP).
 *
 * The filter (Sec. I-A, eqs. (1)-(2)) smooths an image f : Omega -> R^n under
 * the control of a guide p : Omega -> R^rho:
 *     g(i) = sum_{j in W} w(j) phi(p(i-j) - p(i)) f(i-j) / eta(i),
 *     eta(i) = sum_{j in W} w(j) phi(p(i-j) - p(i)),   W = [-S, S]^2,
 * with a Gaussian range kernel phi(x) = exp(-|x|^2 / 2 sigma_r^2) and a
 * Gaussian (bilateral) or box (nonlocal means) spatial kernel w (Sec. III).
 * The library computes the approximation of Algorithm 1 (Sec. II-B): cluster
 * the guide vectors into K centers (bisecting K-means, Sec. II-C), solve the
 * K x K least-squares system of eqs. (11)-(12) once, form the per-pixel
 * weights and coefficients, run the (n+1)K spatial convolutions of
 * eqs. (13)-(14) and recombine per pixel, eqs. (15)-(16).
 *
 * Conventions for every call:
 *  - Images are planar (C, H, W), row-major, FP32, in DEVICE memory of the
 *    context's GPU ("device" below).  "host" marks host memory.
 *  - Window samples outside the image are excluded from both sums (the
 *    convolved images are zero-extended).  Kernels are unnormalised (peak 1).
 *    S is the half-width of the window (W = [-S, S]^2).
 *  - All device work is enqueued on the context's stream.  Calls that return
 *    host results (info, centers, gradients of scalars) synchronise that
 *    stream before returning; the others return with work in flight.
 *  - The caller owns every buffer it passes in.  The library never frees
 *    them.  It keeps its own device workspace inside the context (grown on
 *    demand, freed by fhd_destroy) unless the caller supplies one with
 *    fhd_set_workspace, in which case it allocates no device memory at all.
 *  - Errors are reported through the return value only; nothing is thrown
 *    and nothing aborts across this boundary.  fhd_last_error() gives a
 *    message.  Output contents are unspecified when a call fails.
 *  - Outputs must not alias inputs (FHD_EINVAL where detected); `guide` may
 *    alias `f` (the self-guided bilateral filter).
 */
#ifndef FHD_H
#define FHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fhd_ctx fhd_ctx;

typedef enum {
    FHD_OK = 0,
    FHD_EINVAL = -1,        /* bad argument (sizes, sigmas, NULL, aliasing) */
    FHD_ENOMEM = -2,        /* device/host allocation failed or caller workspace too small */
    FHD_EHIP = -3,          /* a HIP runtime error */
    FHD_ENUMERIC = -4,      /* strict mode: a non-positive normaliser or non-finite output */
    FHD_EUNSUPPORTED = -5   /* valid but outside what this library implements */
} fhd_status;

/* Spatial window omega of eqs. (13)-(14): the Gaussian truncated at the
 * radius, the box, or the recursive Gaussian of Young and van Vliet (1995),
 * the O(1) convolution the paper uses (Sec. II-C): per axis a causal and an
 * anti-causal third-order recursion, each from a zero state at its end of
 * the image, rows then columns; no radius, cost independent of sigma_s
 * (sigma_s >= 0.5; forward filter only: the adjoint and the brute force
 * return FHD_EUNSUPPORTED). */
enum { FHD_SPATIAL_GAUSSIAN = 0, FHD_SPATIAL_BOX = 1, FHD_SPATIAL_YOUNG = 2 };
/* Precision of the point-to-center distance contraction (weights step only;
 * convolutions and normalisation stay FP32). */
enum { FHD_CONTRACT_FP32 = 0, FHD_CONTRACT_BF16 = 1, FHD_CONTRACT_FP16 = 2 };
/* Coefficients: least squares c = A^+ b (eqs. (11)-(12)) or the hard
 * cluster indicator of eq. (17), which gives eq. (18). */
/* Coefficients c(i) of the approximation eq. (9): LSQ, the surrogate fit
 * eq. (11), c = A^+ b(i) (Algorithm 1); HARD, the cluster indicator of
 * eq. (17); EXACT, the per-pixel fit of eq. (10) over the window's own guide
 * samples (fhd_exact_ls; an accuracy study of Sec. II-A: K <= 32, FP32
 * contraction, Gaussian or box window, fhd_filter and fhd_filter_centers
 * only). */
enum { FHD_COEF_LSQ = 0, FHD_COEF_HARD = 1, FHD_COEF_EXACT = 2 };

/* Limits of this library. */
#define FHD_MAX_K 128        /* clusters */
#define FHD_MAX_RHO 64       /* guide dimensions */
#define FHD_MAX_N 64         /* image channels */
#define FHD_MAX_RADIUS 128   /* window half-width S */

typedef struct {
    float sigma_s;        /* Gaussian spatial std (pixels), > 0 (>= 0.5 recursive); ignored for box */
    int radius;           /* S; < 0 means ceil(3 sigma_s) (Sec. III); required (>= 0) for box;
                             ignored for the recursive Gaussian */
    float sigma_r;        /* range std, > 0; +INFINITY allowed (phi == 1) */
    int K;                /* requested clusters, 1..FHD_MAX_K; fewer are used when the
                             guide has fewer distinct vectors (reported as K_eff) */
    int spatial;          /* FHD_SPATIAL_* */
    int contract;         /* FHD_CONTRACT_* */
    int coef;             /* FHD_COEF_* */
    int kmeans_max_iter;  /* 2-means assignment steps per split (default 20) */
    double pinv_rtol;     /* <= 0: singular values above K * s_max * 2^-52 are kept
                             (the MATLAB pinv default); else rtol * s_max */
    int strict;           /* nonzero: FHD_ENUMERIC if a normaliser is <= 0 (or NaN) or an
                             output is not finite (the reduction that fills fhd_info's
                             normaliser fields; synchronises); the outputs are written */
} fhd_params;

/* Diagnostics of one call (host struct, filled when non-NULL). */
typedef struct {
    int K_eff;              /* clusters actually used */
    int pinv_rank;          /* rank kept by the pseudo-inverse */
    int kmeans_rounds;      /* batched split rounds run on the GPU */
    int kmeans_splits;      /* 2-means splits computed (committed or not) */
    double E_K;             /* clustering error, eq. (20) */
    double cond_A;          /* s_max / s_min over the kept singular values of A */
    double pinv_norm;       /* largest |entry| of A^+ */
    float ms_cluster;       /* wall time of the clustering (host clock) */
    float ms_solve;         /* wall time of the K x K solve */
    float ms_filter;        /* wall time from the solve to the end of the filter passes
                               (only when the call synchronises) */
    /* The normaliser r_hat of eq. (16) and the output g_hat = v / r_hat.  The
     * least-squares coefficients can be negative, so r_hat (exactly >= 1 for
     * the filter it approximates) can come out tiny or non-positive; the
     * ratio is not guarded.  Counted on the device by one reduction over the
     * whole output (filter calls only; zero elsewhere). */
    float den_min;          /* smallest r_hat (NaN values are skipped) */
    long long den_nonpos;   /* pixels with r_hat <= 0 or NaN */
    long long den_small;    /* pixels with r_hat < 1e-3 (the non-positive ones included) */
    long long nonfinite;    /* output values that are not finite */
} fhd_info;

/* Fill `p` with defaults: sigma_s 3, radius -1, sigma_r 0.1, K 16, Gaussian,
 * FP32 contraction, least-squares coefficients, 20 iterations, MATLAB pinv
 * tolerance, not strict. */
void fhd_default_params(fhd_params* p);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * to enqueue on (NULL: the null stream).  The stream stays the caller's. */
fhd_status fhd_create(fhd_ctx** ctx, int device, void* hip_stream);
fhd_status fhd_destroy(fhd_ctx* ctx);
fhd_status fhd_set_stream(fhd_ctx* ctx, void* hip_stream);
/* Message of the last failure on this context ("" if none).  Valid until the
 * next call on the context. */
const char* fhd_last_error(const fhd_ctx* ctx);

/* Device workspace (bytes) that fhd_filter needs for one image of this
 * shape with these parameters; it also covers fhd_filter_centers,
 * fhd_cluster and fhd_bruteforce on that image.  The adjoint, batch, volume
 * and approximation-error calls have needs of their own: with a caller
 * workspace that is too small they fail with FHD_ENOMEM (and say so in
 * fhd_last_error); with the library's own workspace it grows as needed. */
fhd_status fhd_workspace_size(const fhd_params* p, int n, int rho, int H, int W,
                              size_t* bytes);
/* Hand the library a caller-owned device buffer of `bytes` bytes (aligned to
 * 256 B) to use as workspace instead of its own; NULL reverts to the
 * library's own.  Calls whose need exceeds it fail with FHD_ENOMEM. */
fhd_status fhd_set_workspace(fhd_ctx* ctx, void* dev, size_t bytes);

/* Intermediates a forward call can keep for its adjoint (the `saved`
 * arguments below).  The adjoint of eqs. (13)-(16) needs, per cluster l,
 * Q_l = w * (c_l [f, 1]) and the coefficients c_l(i) = (A^+ b(i))_l; the
 * forward call forms both (the row-filtered planes of its first pass and the
 * coefficients it computes for them), so a forward call given a saved buffer
 * writes them there, and fhd_filter_backward / fhd_filter_batch_backward
 * given the same buffer skip recomputing them (one row pass and the weights
 * pass).  fhd_saved_size gives the bytes for one image at p->K clusters
 * (K(n+1) planes of (H + 2 radius) x W floats plus K planes of H x W, twice K
 * for guides of more than 8 dimensions or more than 32 clusters);
 * fhd_saved_size_batch for a ragged batch.  Only for what the adjoint
 * covers: FP32 contraction, least-squares coefficients, the Gaussian or box
 * window with radius 1..32, K <= 64 (FHD_EUNSUPPORTED otherwise).
 * The context records which forward call wrote a buffer (the image and guide
 * pointers, shape, window, sigmas and centers); an adjoint call whose
 * arguments differ, or a buffer another call has since overwritten, is
 * rejected with FHD_EINVAL.  The contents of the image and guide are not
 * checked: changing them between the two calls gives the adjoint of the
 * forward call's inputs. */
fhd_status fhd_saved_size(const fhd_params* p, int n, int rho, int H, int W, size_t* bytes);
fhd_status fhd_saved_size_batch(const fhd_params* p, int B, const int* H, const int* W, int n, int rho,
                                size_t* bytes);

/* Step 1 of Algorithm 1: bisecting K-means of the range space eq. (8)
 * (Sec. II-C), on the GPU with FP64 centroid and distance arithmetic.
 * The leaf with the largest SSE (sum of squared distances to its centroid;
 * ties: lower heap id, root 1, children 2h and 2h+1) is split by 2-means
 * seeded with a = the member farthest from the centroid and b = the member
 * farthest from a (ties: lowest pixel index); x joins a's child iff
 * |x - c_a|^2 <= |x - c_b|^2; at most `max_iter` assignment steps, stopping
 * when no label changes.  Splitting stops at K leaves or when no leaf has two
 * distinct members.
 *   guide   device, rho x H x W.
 *   centers host, K x rho FP32, row-major: the K_eff leaf centroids in heap-id
 *           order (rows K_eff..K-1 untouched).
 *   labels  device, H x W int32 cluster index per pixel, or NULL.
 *   K_eff   host, number of clusters produced.
 * Synchronises. */
fhd_status fhd_cluster(fhd_ctx* ctx, const float* guide, int rho, int H, int W, int K,
                       int max_iter, float* centers, int* labels, int* K_eff,
                       fhd_info* info);

/* Step 2 of Algorithm 1 on its own: A_kl = phi(mu_k - mu_l) (eq. (12)) and its
 * pseudo-inverse in FP64 (symmetric eigen-decomposition, singular values
 * |lambda| above the tolerance of fhd_params.pinv_rtol kept).
 *   centers host K x rho FP32;  Apinv host K x K FP64 (row-major), or NULL;
 *   A host K x K FP64 or NULL;  rank host or NULL.
 * FHD_ENUMERIC when the eigen-decomposition does not converge (non-finite
 * centers); every call that solves for A^+ reports the same. */
fhd_status fhd_pinv(const float* centers, int K, int rho, double sigma_r, double rtol,
                    double* A, double* Apinv, int* rank, double* cond);

/* Steps 2-5 of Algorithm 1 with given centers: the K x K solve, the weights
 * b_k(i) = phi(mu_k - p(i)) and coefficients c(i) = A^+ b(i), the
 * convolutions of eqs. (13)-(14) and the recombination of eqs. (15)-(16).
 *   f       device n x H x W;  guide device rho x H x W (may equal f).
 *   centers host K x rho FP32.
 *   out     device n x H x W: g_hat = v / r_hat.
 *   den     device H x W: the normaliser r_hat of eq. (16), or NULL.
 *   labels  device H x W cluster index per pixel; required for FHD_COEF_HARD,
 *           else ignored (may be NULL).
 *   saved   device buffer of saved_bytes (fhd_saved_size) for the adjoint's
 *           intermediates, or NULL (saved_bytes ignored).
 * Returns with the filter in flight unless `info` or strict mode asks for
 * host results. */
fhd_status fhd_filter_centers(fhd_ctx* ctx, const float* f, int n, const float* guide,
                              int rho, int H, int W, const float* centers, int K,
                              const int* labels, const fhd_params* p, float* out,
                              float* den, fhd_info* info, void* saved, size_t saved_bytes);

/* Bytes of device scratch that fhd_filter_centers_noalloc can use. */
#define FHD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* fhd_filter_centers for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and arguments, without `info`, with every device scratch buffer
 * (the intermediate planes, the weight planes, the constants) taken from a
 * static device array of FHD_NOALLOC_SCRATCH_BYTES that each GPU holds until
 * the process ends, and the constants staged through a pinned buffer that
 * fhd_create made.  The call allocates no device or pinned memory and creates
 * no HIP objects (stage timing does not record it).
 *   The caller still passes inputs and outputs.  An image whose scratch need
 *   exceeds FHD_NOALLOC_SCRATCH_BYTES fails with FHD_ENOMEM (fhd_last_error
 *   gives both sizes); K(n+1) planes of (H + 2 radius) x W floats dominate, so
 *   the limit is met e.g. by 256 x 256 RGB with K = 32 and radius 15.
 *   strict: as for fhd_filter_centers (the check's buffers also come from
 *   the scratch; synchronises).
 *   Every call on one GPU shares that GPU's array, which keeps the last call's
 *   contents: calls that overlap on one GPU (contexts on different streams)
 *   race; calls on one context are ordered by its stream. */
fhd_status fhd_filter_centers_noalloc(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int H,
                                      int W, const float* centers, int K, const int* labels, const fhd_params* p,
                                      float* out, float* den);

/* The whole of Algorithm 1: fhd_cluster then fhd_filter_centers.
 *   centers_out host K x rho FP32 (the K_eff centers used), or NULL.
 *   den         device H x W normaliser, or NULL.
 *   saved       device buffer for the adjoint's intermediates (sized by
 *               fhd_saved_size at p->K), or NULL.
 * Synchronises once per clustering round (the greedy split selection runs on
 * the host); returns with the filter passes in flight unless `info` or strict
 * mode asks for host results. */
fhd_status fhd_filter(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho,
                      int H, int W, const fhd_params* p, float* out, float* centers_out,
                      float* den, fhd_info* info, void* saved, size_t saved_bytes);

/* Ragged batch: Algorithm 1 on B independent images of one shape family
 * (n channels, rho guide dimensions, sizes H[b] x W[b]), one clustering tree
 * per image with every clustering pass launched once for all images.
 *   H, W, px_offset host arrays of B; image b holds H[b] * W[b] pixels from
 *           pixel px_offset[b] on; the images are packed back to back
 *           (px_offset[0] = 0, px_offset[b + 1] = px_offset[b] + H[b] W[b]),
 *           otherwise FHD_EINVAL.
 *   f       device: image b is n x H[b] x W[b] planar at element n * px_offset[b].
 *   guide   device: rho x H[b] x W[b] at element rho * px_offset[b] (may equal f).
 *   out     device, laid out like f.  den device, one plane per image at
 *           element px_offset[b], or NULL.
 *   centers_out host B x K x rho (rows K_eff[b]..K-1 of image b untouched) or
 *           NULL;  K_eff host B or NULL;  info host B or NULL.
 *   saved   device buffer for the adjoint's intermediates
 *           (fhd_saved_size_batch), or NULL.
 * Synchronises once per clustering round. */
fhd_status fhd_filter_batch(fhd_ctx* ctx, int B, const int* H, const int* W,
                            const long long* px_offset, const float* f, int n,
                            const float* guide, int rho, const fhd_params* p, float* out,
                            float* centers_out, int* K_eff, float* den, fhd_info* info, void* saved,
                            size_t saved_bytes);

/* Adjoint of fhd_filter_centers for least-squares coefficients (the paper
 * does not differentiate its filter; this is the exact gradient of the
 * computation of Algorithm 1 steps 2-5 for given centers; the clustering
 * that produced them is not differentiated).  Given
 * G = dL/dg_hat it returns dL/df, dL/dguide, dL/dsigma_r, dL/dsigma_s and dL/dmu
 * (the spatial scale enters only through the window omega of eqs. (13)-(14):
 * d omega / d sigma_s = omega |j|^2 / sigma_s^3, radius held fixed); the weights are
 * recomputed from the guide in FP32 (never stored by the forward call), so the
 * gradient is that of the FP32 contraction whatever `p->contract` says.  The
 * sigma_r term through A^+ holds the rank decision of the pseudo-inverse fixed
 * (see fhd_pinv).
 *   f, guide, centers, K, p  as passed to fhd_filter_centers (p->coef must be
 *            FHD_COEF_LSQ; K <= 64; radius 1..32; Gaussian or box window).
 *   out, den device: g_hat and r_hat returned by that forward call.
 *   grad_out device n x H x W: G.
 *   grad_f   device n x H x W output, or NULL.
 *   grad_guide device rho x H x W output, or NULL.  When the guide is the
 *            image (joint filtering of f by itself), dL/df is the sum of the
 *            two outputs.
 *   grad_sigma_r host, one double, or NULL.  Synchronises when non-NULL.
 *   grad_sigma_s host, one double, or NULL (Gaussian window only, else
 *            FHD_EUNSUPPORTED).  Synchronises when non-NULL; costs one more
 *            row pass and column pass and one more K-plane set.
 *   grad_centers host K x rho (FP64), or NULL: dL/dmu with every pixel's
 *            weights b_m(i) = phi(mu_m - p(i)) and A = [phi(mu_k - mu_l)]
 *            differentiated (eq. (12)), the clustering that produced the
 *            centers held fixed.  Synchronises when non-NULL; one more pass
 *            over beta and gamma; FHD_EUNSUPPORTED when its K x K + K(rho+1)
 *            sums exceed the LDS of a block (K = 64 with rho near 64).
 *   saved    the buffer a forward call with these arguments filled (see
 *            fhd_saved_size), or NULL to recompute its contents.
 * Gradient outputs must not alias inputs.  Workspace: five K-plane sets plus
 * the intermediate planes of the forward call. */
fhd_status fhd_filter_backward(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho,
                               int H, int W, const float* centers, int K, const fhd_params* p,
                               const float* out, const float* den, const float* grad_out,
                               float* grad_f, float* grad_guide, double* grad_sigma_r,
                               double* grad_sigma_s, double* grad_centers, const void* saved,
                               size_t saved_bytes);

/* Adjoint of fhd_filter_batch (least-squares coefficients), laid out like
 * it: centers host B x K x rho and K_eff host B as returned by the forward
 * call; out, den its outputs (den required); grad_out, grad_f, grad_guide
 * device in the layouts of f and guide (gradient outputs may be NULL);
 * grad_sigma_r and grad_sigma_s host, the sums over the images, or NULL
 * (synchronise when non-NULL; with grad_sigma_s the images' adjoints run one
 * by one on the auxiliary streams); saved as filled by the forward call, or
 * NULL.  Same limits as fhd_filter_backward. */
fhd_status fhd_filter_batch_backward(fhd_ctx* ctx, int B, const int* H, const int* W,
                                     const long long* px_offset, const float* f, int n,
                                     const float* guide, int rho, const float* centers,
                                     const int* K_eff, const fhd_params* p, const float* out,
                                     const float* den, const float* grad_out, float* grad_f,
                                     float* grad_guide, double* grad_sigma_r, double* grad_sigma_s,
                                     const void* saved, size_t saved_bytes);

/* The brute-force filter of eqs. (1)-(2) on the GPU (FP32), the reference
 * the approximation is measured against.  out device n x H x W; den device
 * H x W (eta) or NULL. */
fhd_status fhd_bruteforce(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho,
                          int H, int W, const fhd_params* p, float* out, float* den);

/* The guide of nonlocal means (Sec. I-A; PCA of patches as in Sec. III-C):
 * every pixel's patch x (patch x patch x n values, half-sample symmetric
 * extension at the borders, flattened in (dy, dx, channel) order) is
 * projected onto the `dims` leading eigenvectors of the patch covariance
 * (1/N normalised, FP64 on the host):  guide_d(i) = sum_j (x_j(i) - mean_j) V_jd.
 * Each eigenvector's largest-magnitude component is made positive.
 *   f        device n x H x W;  patch odd, patch*patch*n <= 160;
 *   dims     1 .. min(patch*patch*n, FHD_MAX_RHO);
 *   guide    device dims x H x W (output);
 *   eigvals  host, patch*patch*n covariance eigenvalues in descending order, or NULL.
 * Synchronises (the eigen-decomposition runs on the host between kernels). */
fhd_status fhd_nlm_guide(fhd_ctx* ctx, const float* f, int n, int H, int W, int patch, int dims,
                         float* guide, double* eigvals);

/* All of Algorithm 1 on a 3-D domain (the flow-field denoising of Sec. III-F
 * filters a volume): the bisecting K-means of the voxels' guide vectors (all
 * D H W voxels as one set, in (z, y, x) order), A and A^+, the weights and
 * coefficients per voxel, the (n+1)K convolutions over the window
 * [-S,S]^3 with omega(j) = exp(-|j|^2 / 2 sigma_s^2) (or 1, box), voxels
 * outside the volume left out, and the recombination of eqs. (15)-(16).
 *   f      device n x D x H x W;  guide device rho x D x H x W (may alias f);
 *   out    device n x D x H x W;  den device D x H x W or NULL;
 *   centers_out  host K x rho or NULL;  info or NULL.
 * The parameters as for fhd_filter, limited to the Gaussian or box window
 * and the FP32 contraction (FHD_EUNSUPPORTED otherwise); coef selects least
 * squares or the hard variant of eqs. (17)-(18); D * H <= 65535.  Enqueued on the context's stream; the
 * clustering synchronises as in fhd_filter. */
fhd_status fhd_filter_volume(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int D, int H, int W,
                             const fhd_params* p, float* out, float* centers_out, float* den, fhd_info* info);

/* Eqs. (1)-(2) on a 3-D domain, directly (the comparator of
 * fhd_filter_volume): window [-S,S]^3, omega(j) = exp(-|j|^2 / 2 sigma_s^2)
 * (the product of the 1-D taps) or 1, neighbours outside the volume left out.
 * Arguments as for fhd_filter_volume (no clustering parameters used); FP32,
 * cost (2S+1)^3 (rho + n) per voxel.  Enqueued on the context's stream. */
fhd_status fhd_bruteforce_volume(fhd_ctx* ctx, const float* f, int n, const float* guide, int rho, int D, int H,
                                 int W, const fhd_params* p, float* out, float* den);

/* Eq. (10) solved at every pixel (Sec. II-A): the coefficients c*(i) of
 * the least-squares fit
 *   min_c sum_q (phi(p(q) - p(i)) - sum_k c_k phi(p(q) - mu_k))^2,
 * q over the in-image pixels of the (2S+1)^2 window around i (Theta_i of
 * eq. (10), with multiplicity), taken as the minimum-norm minimiser M_i^+ y_i
 * of the window's design matrix (rows b(q), targets phi(p(q) - p(i))), with
 * singular values at or below max(m, K) 2^-52 s_max dropped (the tolerance
 * of the MATLAB pinv), m the window's in-image pixels.  The paper fits over
 * the centers instead (eq. (11)) to share one K x K pseudo-inverse across
 * all pixels; this call gives the fit it approximates, and the objective of
 * eq. (10) at both.
 *   guide    device rho x H x W;  centers host K x rho FP32, 1 <= K <= 32;
 *   p        sigma_r, pinv_rtol (for A^+ in obj11) and the window as in
 *            fhd_approx_error (the recursive Gaussian is rejected);
 *   coef     device K x H x W FP32 (plane k = c*_k over the image) or NULL;
 *   obj      device H x W FP32: the minimum of eq. (10), or NULL;
 *   obj11    device H x W FP32: eq. (10) at c = A^+ b(i), or NULL.
 * At least one output.  FP64 throughout (a streaming Givens QR of the
 * design matrix and a Jacobi SVD of its K x K triangle, per pixel); cost
 * ~ (2S+1)^2 K^2 per pixel.  Enqueued on the context's stream. */
fhd_status fhd_exact_ls(fhd_ctx* ctx, const float* guide, int rho, int H, int W, const float* centers, int K,
                        const fhd_params* p, float* coef, float* obj, float* obj11);

/* Clusters used (K_eff) by the last call on this context that clustered
 * (fhd_filter, fhd_filter_volume, fhd_cluster, fhd_filter_batch: its last
 * image); 0 before any.  A caller that only wants the number of centers
 * fhd_filter wrote can skip fhd_info, whose normaliser fields cost one device
 * reduction and a synchronisation. */
int fhd_last_k_eff(const fhd_ctx* ctx);

/* Error of the kernel approximation at each pixel's own samples (Sec. II-A):
 * the objective of eq. (10) evaluated at the coefficients the method uses,
 * c(i) = A^+ b(i) of eqs. (11)-(12),
 *   err[i] = sum_{q} (phi(p(q) - p(i)) - sum_k c_k(i) phi(p(q) - mu_k))^2,
 * q over the in-image pixels of the (2S+1)^2 window around i (the set Theta_i
 * of eq. (10), counted with multiplicity).  Its pixel mean is the averaged
 * least-squares error (a script E indexed by K in Sec. II-A, written E_ls
 * here; not the clustering error E_K of eq. (20)) whose fall with K the
 * paper plots.
 *   guide    device rho x H x W;  centers host K x rho FP32, 1 <= K <= 64;
 *   p        sigma_r, pinv_rtol and the window: radius (or ceil(3 sigma_s)
 *            when radius < 0, Gaussian), box needs radius >= 0; the recursive
 *            Gaussian is rejected (no finite window);
 *   err      device H x W FP32 (output) or NULL;
 *   mean     host, E_ls (FP64 sum of the per-pixel FP64 sums / N) or NULL;
 *            when given the call synchronises.  At least one of the two.
 * Terms are FP32 and sums FP64.  Cost ~ K (2S+1)^2 (rho + 1) per pixel. */
fhd_status fhd_approx_error(fhd_ctx* ctx, const float* guide, int rho, int H, int W, const float* centers, int K,
                            const fhd_params* p, float* err, double* mean);

/* Anisotropic Gaussian range kernel (Sec. III: one experiment, the low-light
 * denoising of Sec. III-E, uses a separate sigma_r per guide dimension):
 *   phi(x) = exp(-sum_d x_d^2 / (2 sigma_d^2)).
 * It equals the isotropic kernel with sigma_r = 1 on the guide scaled per
 * dimension, so this call writes
 *   out[d][i] = guide[d][i] / sigma_d      (FP32, correctly rounded)
 * and every other entry point, given `out` and sigma_r = 1, filters with the
 * anisotropic kernel; clustering and centers are then in the scaled units.
 * The map is diagonal and linear, so the same call turns dL/d(out) into
 * dL/d(guide).
 *   guide, out  device rho x N (planar), N >= 0 (may be NULL when N == 0);
 *               out == guide is allowed (in place), any other overlap is
 *               rejected;
 *   sigma_d     host array of rho finite values > 0;  1 <= rho <= FHD_MAX_RHO.
 * Enqueued on the context's stream; does not synchronise. */
fhd_status fhd_scale_guide(fhd_ctx* ctx, const float* guide, int rho, long long N, const float* sigma_d,
                           float* out);

/* Stage timing with HIP events on the context's stream (for benchmarks).
 * While enabled, every call records an event pair around each stage's
 * kernels; fhd_timing_read returns, per stage, the summed elapsed
 * milliseconds and the number of kernel launches between the recorded pairs
 * since the last read, then forgets them (it synchronises the stream).
 * Stages: */
enum {
    FHD_STAGE_CLUSTER = 0,  /* all clustering kernels of one call (first to last) */
    FHD_STAGE_WEIGHTS = 1,  /* weights pass (materialised b and c planes) */
    FHD_STAGE_ROW = 2,      /* row pass of the convolutions */
    FHD_STAGE_COL = 3,      /* column pass with the recombination */
    FHD_STAGE_BRUTE = 4,    /* brute force */
    FHD_STAGE_LLOYD = 5,    /* the 2-means assignment steps of the clustering (inside
                               FHD_STAGE_CLUSTER): one event pair around each round's
                               chain of kmeans_max_iter launches */
    FHD_NUM_STAGES = 6
};
fhd_status fhd_timing_enable(fhd_ctx* ctx, int enable);
/* ms and launches: host arrays of FHD_NUM_STAGES entries. */
fhd_status fhd_timing_read(fhd_ctx* ctx, double* ms, int* launches);
/* Algorithmic work per stage recorded while timing is enabled, since the
 * last call (host array of FHD_NUM_STAGES; then reset): for FHD_STAGE_LLOYD
 * the guide points streamed by the assignment steps (a job's points once per
 * step it ran before stopping), 0 for the other stages. */
fhd_status fhd_timing_units(fhd_ctx* ctx, long long* units);

#ifdef __cplusplus
}
#endif

#endif /* FHD_H */
