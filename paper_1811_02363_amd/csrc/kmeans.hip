// Bisecting K-means of the range space (Algorithm 1, step 1; Sec. II-C) on
// the GPU.
//
// Design.  The guide vectors are packed point-major (AoS) with their pixel
// index, and every cluster is a contiguous range of that array (two ping-pong
// copies; a split stably partitions its range into the other copy).  Splits
// are computed in batched rounds: each round computes the 2-means split of
// every leaf the greedy largest-SSE rule may still pick (seeds, assignment
// steps, children's SSE, partition), one launch per pass for all of them.
// The host commits splits greedily between rounds; that is the only host
// synchronisation, once per round.
//
// Passes stream the member points once and write one partial record per
// block; a one-block-per-job finalize kernel reduces the records and updates
// the job's state.  Labels are never stored: the assignment is a pure
// function of the point and the job's two centers, so the pass that needs the
// final labels (split statistics, partition) recomputes them bit for bit.
//
// Arithmetic: distances and centroid sums in FP64 from the FP32 points, in a
// fixed reduction order (per lane sequential, fixed shuffle tree, waves in
// order, blocks in order), so a run is deterministic.  No floating-point
// atomics.  Lanes are laid out LP per point, each lane holding D consecutive
// dimensions (LP = 1 for rho <= 8).  Points are packed at a stride of LP * D
// floats with the dimensions beyond rho set to zero (centers too), so every
// load is unconditional and the padded terms add exactly 0.0 to distances.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>

#include "fhd_internal.h"

namespace fhd {
namespace {

constexpr int KT = 256;          // threads per block
constexpr int KWAVES = KT / 64;  // waves per block
constexpr int FT = 256;          // threads per finalize block
static_assert(FT == KT, "the assignment step runs the finalize reduction with its own threads");
constexpr int KITERS = 16;       // point groups per block and pass
constexpr int DPL = 8;           // dimensions per lane (at most)
// points per lane group in flight per step: eight for one lane of up to four
// dimensions per point, else four (register budget)
template <int D>
constexpr int unr() { return D <= 4 ? 8 : 4; }
// the assignment step stages its points as FP32 (converted at use): sixteen
// points per lane group in flight for up to four dimensions, else eight
template <int D>
constexpr int unr_lloyd() { return D <= 4 ? 16 : 8; }

// per-job integer state
enum { JI_START, JI_COUNT, JI_BUF, JI_FIRST, JI_NBLK, JI_NA, JI_W = 8 };
// per-job FP64 results
enum { JD_SSEA, JD_SSEB, JD_NA, JD_NB, JD_SPLA, JD_SPLB, JD_STEPS, JD_W = 7 };

struct KmArgs {
    float* pts[2];
    int* idx[2];
    const int4* btab;  // per block: job (bit 30: its point buffer), first point, point count,
                       // rank within job (or label)
    int* blkA;         // per block: members of the first child (split pass)
    double* part;      // per block records, entry-major: entry e of block b at part[e * pst + b]
    double* part2;     // the same for the odd assignment steps
    int* ji;           // per job ints, JI_W each
    double* jm;        // per job centroid (rho)
    double* ca;        // per job current centers (first / second child), rho each
    double* cb;
    double* cst;       // assignment-step centers, three generations: (ca, cb) of job j for step t
                       // at cst[((t % 3) * mj + j) * 2 rho]
    int* jstop;        // per job, two generations: stopped before step t at jstop[(t & 1) * mj + j]
    int mj;            // job capacity
    double* fa;        // per job centers whose assignment gives the final labels
    double* fb;
    double* jd;        // per job results, JD_W each
    int rho;
    long long pst;     // record entry stride (the block capacity)
    int ps;            // point stride in floats (LP * D of the launched layout)
};

// ---------------------------------------------------------------------------
// lane layout

template <int LP, int D>
struct Lanes {
    static constexpr int PPW = 64 / LP;  // points per wave
    int lane, wave, sub, pw, d0;
    __device__ Lanes() {
        lane = threadIdx.x & 63;
        wave = threadIdx.x >> 6;
        sub = lane & (LP - 1);
        pw = lane / LP;
        d0 = sub * D;
    }
};

// this lane's dimensions of point `pos` (stored zeros beyond rho)
template <int LP, int D>
__device__ __forceinline__ void load_dims(const float* pts, long long pos, int d0, double (&x)[D]) {
    const float* p = pts + pos * (LP * D) + d0;
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = (double)p[k];
}

template <int LP, int D>
__device__ __forceinline__ void load_dims_f(const float* pts, long long pos, int d0, float (&x)[D]) {
    const float* p = pts + pos * (LP * D) + d0;
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = p[k];
}

constexpr int JOB_BITS = 0x3fffffff;
__device__ __forceinline__ int bjob(int4 bt) { return bt.x & JOB_BITS; }
__device__ __forceinline__ int bbuf(int4 bt) { return bt.x >> 30; }

template <int D>
__device__ __forceinline__ void load_center(const double* c, int rho, int d0, double (&v)[D]) {
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = (d0 + k < rho) ? c[d0 + k] : 0.0;
}

// |x - c|^2 over the point's dimensions: sequential over a lane's dimensions
// (separately rounded products and sums), then a shuffle tree over its LP lanes.
template <int LP, int D>
__device__ __forceinline__ double dist2(const double (&x)[D], const double (&c)[D], int rho, int d0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {  // beyond rho: (0 - 0)^2 added to s >= +0 leaves s unchanged
        const double t = __dsub_rn(x[k], c[k]);
        s = __dadd_rn(s, __dmul_rn(t, t));
    }
#pragma unroll
    for (int o = 1; o < LP; o <<= 1) s = __dadd_rn(s, __shfl_xor(s, o, 64));
    return s;
}

// The assignment rule: first child iff |x - c_a|^2 <= |x - c_b|^2.
template <int LP, int D>
__device__ __forceinline__ bool to_first(const double (&x)[D], const double (&a)[D], const double (&b)[D], int rho,
                                         int d0) {
    return dist2<LP, D>(x, a, rho, d0) <= dist2<LP, D>(x, b, rho, d0);
}

// One block's record: entry e at p[e * st].
struct RecRef {
    double* p;
    long long st;
    __device__ double& operator[](int e) const { return p[(long long)e * st]; }
    __device__ RecRef operator+(int o) const { return RecRef{p + (long long)o * st, st}; }
};

template <int OP>
__device__ __forceinline__ double op2(double u, double v) {
    return OP == 0 ? u + v : (OP == 1 ? fmin(u, v) : fmax(u, v));
}

// Block reduction of per-lane dimension values (lanes with equal `sub` hold
// the same dimensions); thread t < rho writes the total of dimension t to out[t].
template <int LP, int D, int OP>
__device__ __forceinline__ void block_dims(double (&v)[D], double (*red)[64], int rho, RecRef out) {
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int o = LP; o < 64; o <<= 1) v[k] = op2<OP>(v[k], __shfl_xor(v[k], o, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane < LP)
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (lane * D + k < 64) red[wave][lane * D + k] = v[k];
    __syncthreads();
    if (threadIdx.x < rho) {
        double r = red[0][threadIdx.x];
        for (int q = 1; q < KWAVES; ++q) r = op2<OP>(r, red[q][threadIdx.x]);
        out[threadIdx.x] = r;
    }
}

// Sum over every lane of the block, result in thread 0.
__device__ __forceinline__ double block_sum(double v, double (*red)[64]) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave][0] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < KWAVES; ++q) r += red[q][0];
    return r;
}

// The assignment step's block record [sumA (rho), sumB (rho), nA, nB] in one
// LDS round: per value the shuffle tree and the wave order of block_dims and
// block_sum, so the same sums bit for bit.
template <int LP, int D>
__device__ __forceinline__ void block_lloyd_record(double (&sa)[D], double (&sb)[D], double na, double nb,
                                                   double (*red)[2 * 64 + 2], int rho, RecRef out) {
    constexpr int LPD = LP * D;
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int o = LP; o < 64; o <<= 1) {
            sa[k] += __shfl_xor(sa[k], o, 64);
            sb[k] += __shfl_xor(sb[k], o, 64);
        }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        na += __shfl_xor(na, o, 64);
        nb += __shfl_xor(nb, o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < LP)
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (lane * D + k < 64) {
                red[wave][lane * D + k] = sa[k];
                red[wave][LPD + lane * D + k] = sb[k];
            }
    if (lane == 0) {
        red[wave][2 * LPD] = na;
        red[wave][2 * LPD + 1] = nb;
    }
    __syncthreads();
    const int e = threadIdx.x;
    if (e < 2 * rho + 2) {
        const int src = e < rho ? e : (e < 2 * rho ? LPD + e - rho : 2 * LPD + e - 2 * rho);
        double r = red[0][src];
        for (int q = 1; q < KWAVES; ++q) r += red[q][src];
        out[e] = r;
    }
}

// Finalize helper: res[e] = reduction over the job's blocks of record entry
// e0 + e, for e < E, with the operation opof(e) (0 sum, 1 min, 2 max).  A
// fixed order: a power-of-two group of G threads per entry; thread `sub` of a
// group folds records sub, sub + G, sub + 2G, ... (adjacent threads read
// adjacent blocks' entries; sixteen loads in flight)
// into four partials by slot (q mod 4), combined as (p0 op p1) op (p2 op p3);
// then a pairwise tree over the group.  Called by all FT threads.
template <class OpOf>
__device__ void reduce_records(const double* part, int first, int nblk, long long pst, int e0, int E, OpOf opof,
                               double* tmp, double* res) {
    auto ident = [](int op) { return op == 0 ? 0.0 : (op == 1 ? INFINITY : -INFINITY); };
    auto fold = [](int op, double u, double v) { return op == 0 ? u + v : (op == 1 ? fmin(u, v) : fmax(u, v)); };
    for (int base = 0; base < E; base += FT) {
        const int Ec = min(FT, E - base);
        const int G = 1 << (31 - __clz(FT / Ec));  // threads per entry, a power of two
        const int t = threadIdx.x;
        const bool act = t < Ec * G;
        const int e = base + t / G, sub = t & (G - 1);
        const int op = act ? opof(e) : 0;
        const double id = ident(op);
        double acc = id;
        if (act) {
            double p[4] = {id, id, id, id};
            const double* r = part + (long long)(e0 + e) * pst + first + sub;
            for (int b = sub; b < nblk; b += 16 * G, r += 16 * G) {
                double w[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) w[q] = b + q * G < nblk ? r[q * G] : id;
#pragma unroll
                for (int q = 0; q < 16; ++q) p[q & 3] = fold(op, p[q & 3], w[q]);
            }
            acc = fold(op, fold(op, p[0], p[1]), fold(op, p[2], p[3]));
        }
        // pairwise tree over the group: levels of 64 and more through LDS,
        // the rest within the wave by shuffles (the same pairs, so the same
        // sums); a group of at most 64 threads lies in one wave
        double v = acc;
        int h = G >> 1;
        if (G > 64) {
            tmp[t] = v;
            __syncthreads();
            for (; h >= 64; h >>= 1) {
                if (act && sub < h) tmp[t] = fold(op, tmp[t], tmp[t + h]);
                __syncthreads();
            }
            v = tmp[t];
        }
        for (; h >= 1; h >>= 1) {
            const double o = __shfl_down(v, h, 64);
            if (sub < h) v = fold(op, v, o);
        }
        if (act && sub == 0) res[base + t / G] = v;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// passes

// Points of one image (planar rho x N guide) into the packed array from
// position `base` on; idx holds the position in the concatenation of images.
__global__ __launch_bounds__(KT) void km_pack(const float* __restrict__ guide, int rho, int ps, long long N,
                                              long long base, float* __restrict__ pts, int* __restrict__ idx) {
    const long long i = (long long)blockIdx.x * KT + threadIdx.x;
    if (i >= N) return;
    for (int d = 0; d < ps; ++d) pts[(base + i) * ps + d] = d < rho ? guide[(long long)d * N + i] : 0.0f;
    idx[base + i] = (int)(base + i);
}

// Member sums and per-dimension min/max.  Record: sum[rho], min[rho], max[rho].
template <int LP, int D>
__global__ __launch_bounds__(KT) void km_stats(KmArgs a) {
    __shared__ double red[KWAVES][64];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bjob(bt), s = bt.y, cnt = bt.z;
    const float* pts = a.pts[a.ji[job * JI_W + JI_BUF]];
    const int rho = a.rho;
    const Lanes<LP, D> L;
    double sum[D], mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        sum[k] = 0.0;
        mn[k] = INFINITY;
        mx[k] = -INFINITY;
    }
    for (int base = 0; base < cnt; base += KWAVES * L.PPW) {
        const int p = base + L.wave * L.PPW + L.pw;
        if (p >= cnt) continue;
        double x[D];
        load_dims<LP, D>(pts, s + p, L.d0, x);
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (L.d0 + k < rho) {
                sum[k] += x[k];
                mn[k] = fmin(mn[k], x[k]);
                mx[k] = fmax(mx[k], x[k]);
            }
    }
    const RecRef rec{a.part + blockIdx.x, a.pst};
    block_dims<LP, D, 0>(sum, red, rho, rec);
    block_dims<LP, D, 1>(mn, red, rho, rec + rho);
    block_dims<LP, D, 2>(mx, red, rho, rec + 2 * rho);
}

// SSE of the whole job around its centroid jm.  Record: sse.
template <int LP, int D>
__global__ __launch_bounds__(KT) void km_sse1(KmArgs a) {
    __shared__ double red[KWAVES][64];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bjob(bt), s = bt.y, cnt = bt.z;
    const float* pts = a.pts[a.ji[job * JI_W + JI_BUF]];
    const int rho = a.rho;
    const Lanes<LP, D> L;
    double c[D];
    load_center(a.jm + job * rho, rho, L.d0, c);
    double e = 0.0;
    for (int base = 0; base < cnt; base += KWAVES * L.PPW) {
        const int p = base + L.wave * L.PPW + L.pw;
        if (p >= cnt) continue;
        double x[D];
        load_dims<LP, D>(pts, s + p, L.d0, x);
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (L.d0 + k < rho) {
                const double t = x[k] - c[k];
                e += t * t;
            }
    }
    const double tot = block_sum(e, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
}

// Seed search: the member farthest from the centroid (which == 0) or from the
// first seed (which == 1); ties -> lowest pixel index.  Record: d, pixel, pos.
template <int LP, int D>
__global__ __launch_bounds__(KT) void km_far(KmArgs a, int which) {
    __shared__ double rb[KWAVES];
    __shared__ int ri[KWAVES], rp[KWAVES];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bjob(bt), s = bt.y, cnt = bt.z;
    const int buf = a.ji[job * JI_W + JI_BUF];
    const float* pts = a.pts[buf];
    const int* idx = a.idx[buf];
    const int rho = a.rho;
    const Lanes<LP, D> L;
    double r[D];
    load_center((which == 0 ? a.jm : a.ca) + job * rho, rho, L.d0, r);
    double best = -1.0;
    int bidx = INT_MAX, bpos = -1;
    for (int base = 0; base < cnt; base += unr<D>() * KWAVES * L.PPW) {
        constexpr int UNR = unr<D>();
        double x[UNR][D];
        int pp[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            pp[u] = base + (u * KWAVES + L.wave) * L.PPW + L.pw;
            load_dims<LP, D>(pts, pp[u] < cnt ? s + pp[u] : s, L.d0, x[u]);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const double t = dist2<LP, D>(x[u], r, rho, L.d0);
            if (pp[u] < cnt) {
                const int pi = idx[s + pp[u]];
                if (t > best || (t == best && pi < bidx)) {
                    best = t;
                    bidx = pi;
                    bpos = s + pp[u];
                }
            }
        }
    }
#pragma unroll
    for (int o = LP; o < 64; o <<= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bidx, o, 64);
        const int op = __shfl_xor(bpos, o, 64);
        if (ob > best || (ob == best && oi < bidx)) {
            best = ob;
            bidx = oi;
            bpos = op;
        }
    }
    if (L.lane == 0) {
        rb[L.wave] = best;
        ri[L.wave] = bidx;
        rp[L.wave] = bpos;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < KWAVES; ++q)
            if (rb[q] > best || (rb[q] == best && ri[q] < bidx)) {
                best = rb[q];
                bidx = ri[q];
                bpos = rp[q];
            }
        const RecRef rec{a.part + blockIdx.x, a.pst};
        rec[0] = best;
        rec[1] = (double)bidx;
        rec[2] = (double)bpos;
    }
}

// The 2-means state machine after assignment step `st` (labels L_st from the
// centers c_st; m = means of L_st, from the step's records in `res`):
//   a child would be empty   -> stop; final labels L_{st-1} (centers c_{st-1});
//   m equals c_st, st >= 1   -> converged; final labels L_st (centers c_st);
//   otherwise                -> c_{st+1} = m; after max_iter steps stop with
//                               final labels L_st (centers c_st).
// Equal means from a fixed summation order follow from equal labels, and
// equal means make the next assignment repeat the current one, so this stops
// with the labels and centers of the label-change rule.  Returns 0, 1, 2 for
// the three cases (one thread).
__device__ __forceinline__ int lloyd_act(const double* res, const double* c, int rho, int st) {
    const double NA = res[2 * rho], NB = res[2 * rho + 1];
    if (NA == 0.0 || NB == 0.0) return 0;
    bool same = st >= 1;
    for (int t = 0; t < rho && same; ++t) same = (res[t] / NA == c[t]) && (res[rho + t] / NB == c[rho + t]);
    return same ? 1 : 2;
}

// The job's final state after it stops at the decision on step `st`: the
// centers whose assignment gives the final labels (fa, fb) and the children's
// centroids (ca, cb).  Threads < rho.
__device__ __forceinline__ void lloyd_final(const KmArgs& a, int job, int act, int st, const double* res) {
    const int rho = a.rho, t = threadIdx.x;
    if (t == 0) a.jd[job * JD_W + JD_STEPS] = st + 1;  // assignment steps that streamed the job's points
    if (t >= rho) return;
    const double* c = a.cst + ((long long)(st % 3) * a.mj + job) * 2 * rho;             // c_st
    const double* l = a.cst + ((long long)((st + 2) % 3) * a.mj + job) * 2 * rho;       // c_{st-1}
    const double* f = act == 0 && st >= 1 ? l : c;
    a.fa[job * rho + t] = f[t];
    a.fb[job * rho + t] = f[rho + t];
    if (act == 2) {
        a.ca[job * rho + t] = res[t] / res[2 * rho];
        a.cb[job * rho + t] = res[rho + t] / res[2 * rho + 1];
    } else {
        a.ca[job * rho + t] = c[t];
        a.cb[job * rho + t] = c[rho + t];
    }
}

// Assignment step t of every running job.  From the second step on, every
// block first reduces its job's records of step t - 1 and takes the state
// machine's decision itself (the same fixed-order sums in every block, so the
// same decision and centers); the job's first block records the outcome.
// Record: sumA[rho], sumB[rho], nA, nB.
template <int LP, int D>
__global__ __launch_bounds__(KT) void km_lloyd(KmArgs a, int t) {
    __shared__ double red[KWAVES][2 * 64 + 2];
    __shared__ double tmp[KT];
    __shared__ double res[2 * FHD_MAX_RHO + 2];
    __shared__ double cen[2 * FHD_MAX_RHO];
    __shared__ double cpv[2 * FHD_MAX_RHO];
    __shared__ int s_act;
    const int4 bt = a.btab[blockIdx.x];
    const int job = bjob(bt), s = bt.y, cnt = bt.z, rank = bt.w;
    const int rho = a.rho;
    const bool lead = rank == 0;
    int* stop_now = a.jstop + (long long)(t & 1) * a.mj + job;
    double* cnow = a.cst + ((long long)(t % 3) * a.mj + job) * 2 * rho;
    if (t > 0) {
        // The stop flag, the job's block count and the previous centers are
        // fetched together; a job's blocks are contiguous in the block table,
        // so its first block is this block's index less its rank.
        const int nblk = a.ji[job * JI_W + JI_NBLK];
        const int stopped = a.jstop[(long long)((t - 1) & 1) * a.mj + job];
        const double* cprev = a.cst + ((long long)((t - 1) % 3) * a.mj + job) * 2 * rho;
        const double cp = threadIdx.x < 2 * rho ? cprev[threadIdx.x] : 0.0;
        if (stopped | (nblk < 0)) {  // (nblk is never negative: the test keeps its load ahead of the branch)
            if (lead && threadIdx.x == 0) *stop_now = 1;
            return;
        }
        reduce_records((t - 1) & 1 ? a.part2 : a.part, (int)blockIdx.x - rank, nblk, a.pst, 0, 2 * rho + 2,
                       [](int) { return 0; }, tmp, res);
        if (threadIdx.x < 2 * rho) cpv[threadIdx.x] = cp;
        __syncthreads();
        if (threadIdx.x == 0) s_act = lloyd_act(res, cpv, rho, t - 1);
        __syncthreads();
        const int act = s_act;
        if (act != 2) {
            if (lead) {
                lloyd_final(a, job, act, t - 1, res);
                if (threadIdx.x == 0) *stop_now = 1;
            }
            return;
        }
        if (threadIdx.x < 2 * rho)
            cen[threadIdx.x] = threadIdx.x < rho ? res[threadIdx.x] / res[2 * rho]
                                                 : res[threadIdx.x] / res[2 * rho + 1];
        __syncthreads();
        if (lead) {
            if (threadIdx.x < 2 * rho) cnow[threadIdx.x] = cen[threadIdx.x];
            if (threadIdx.x == 0) *stop_now = 0;
        }
    } else {
        if (threadIdx.x < 2 * rho) cen[threadIdx.x] = cnow[threadIdx.x];
        if (lead && threadIdx.x == 0) *stop_now = 0;
        __syncthreads();
    }
    const float* pts = a.pts[bbuf(bt)];
    const Lanes<LP, D> L;
    double ca[D], cb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ca[k] = L.d0 + k < rho ? cen[L.d0 + k] : 0.0;
        cb[k] = L.d0 + k < rho ? cen[rho + L.d0 + k] : 0.0;
    }
    double sa[D], sb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) sa[k] = sb[k] = 0.0;
    double na = 0.0, nb = 0.0;
    constexpr int UNR = unr_lloyd<D>();
    for (int base = 0; base < cnt; base += UNR * KWAVES * L.PPW) {
        float x[UNR][D];
        bool valid[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int p = base + (u * KWAVES + L.wave) * L.PPW + L.pw;
            valid[u] = p < cnt;
            load_dims_f<LP, D>(pts, valid[u] ? s + p : s, L.d0, x[u]);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            double xd[D];
#pragma unroll
            for (int k = 0; k < D; ++k) xd[k] = (double)x[u][k];
            const bool A = to_first<LP, D>(xd, ca, cb, rho, L.d0);
            if (valid[u]) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    if (A) sa[k] += xd[k];
                    else sb[k] += xd[k];
                }
                if (L.sub == 0) {
                    if (A) na += 1.0;
                    else nb += 1.0;
                }
            }
        }
    }
    const RecRef rec{(t & 1 ? a.part2 : a.part) + blockIdx.x, a.pst};
    block_lloyd_record<LP, D>(sa, sb, na, nb, red, rho, rec);
}

// Final labels (assignment with fa, fb): per child member count, SSE around
// the child's centroid (ca / cb) and per-dimension min/max.
// Record: sseA, sseB, nA, nB, minA[rho], maxA[rho], minB[rho], maxB[rho].
template <int LP, int D>
__global__ __launch_bounds__(KT) void km_split(KmArgs a) {
    __shared__ double red[KWAVES][64];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bjob(bt), s = bt.y, cnt = bt.z;
    const float* pts = a.pts[a.ji[job * JI_W + JI_BUF]];
    const int rho = a.rho;
    const Lanes<LP, D> L;
    double fa[D], fb[D], ma[D], mb[D];
    load_center(a.fa + job * rho, rho, L.d0, fa);
    load_center(a.fb + job * rho, rho, L.d0, fb);
    load_center(a.ca + job * rho, rho, L.d0, ma);
    load_center(a.cb + job * rho, rho, L.d0, mb);
    double lo_a[D], hi_a[D], lo_b[D], hi_b[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo_a[k] = lo_b[k] = INFINITY;
        hi_a[k] = hi_b[k] = -INFINITY;
    }
    double ea = 0.0, eb = 0.0, na = 0.0, nb = 0.0;
    for (int base = 0; base < cnt; base += unr<D>() * KWAVES * L.PPW) {
        constexpr int UNR = unr<D>();
        double x[UNR][D];
        bool valid[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int p = base + (u * KWAVES + L.wave) * L.PPW + L.pw;
            valid[u] = p < cnt;
            load_dims<LP, D>(pts, valid[u] ? s + p : s, L.d0, x[u]);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const bool A = to_first<LP, D>(x[u], fa, fb, rho, L.d0);
            if (!valid[u]) continue;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                if (L.d0 + k >= rho) continue;
                if (A) {
                    const double t = x[u][k] - ma[k];
                    ea += t * t;
                    lo_a[k] = fmin(lo_a[k], x[u][k]);
                    hi_a[k] = fmax(hi_a[k], x[u][k]);
                } else {
                    const double t = x[u][k] - mb[k];
                    eb += t * t;
                    lo_b[k] = fmin(lo_b[k], x[u][k]);
                    hi_b[k] = fmax(hi_b[k], x[u][k]);
                }
            }
            if (L.sub == 0) {
                if (A) na += 1.0;
                else nb += 1.0;
            }
        }
    }
    const RecRef rec{a.part + blockIdx.x, a.pst};
    const double tea = block_sum(ea, red);
    const double teb = block_sum(eb, red);
    const double tna = block_sum(na, red);
    const double tnb = block_sum(nb, red);
    if (threadIdx.x == 0) {
        rec[0] = tea;
        rec[1] = teb;
        rec[2] = tna;
        rec[3] = tnb;
        a.blkA[blockIdx.x] = (int)tna;
    }
    block_dims<LP, D, 1>(lo_a, red, rho, rec + 4);
    block_dims<LP, D, 2>(hi_a, red, rho, rec + 4 + rho);
    block_dims<LP, D, 1>(lo_b, red, rho, rec + 4 + 2 * rho);
    block_dims<LP, D, 2>(hi_b, red, rho, rec + 4 + 3 * rho);
}

// Stable partition of each job's range by the final labels into the other
// copy: first-child members first, both groups in their original order.
template <int LP, int D>
__global__ __launch_bounds__(KT) void km_scatter(KmArgs a) {
    __shared__ int red[KWAVES];
    __shared__ int s_offA, s_offB, s_wa[KWAVES], s_wb[KWAVES];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bjob(bt), s = bt.y, cnt = bt.z, rank = bt.w;
    const int* ji = a.ji + job * JI_W;
    const int buf = ji[JI_BUF];
    const float* src = a.pts[buf];
    const int* isrc = a.idx[buf];
    float* dst = a.pts[1 - buf];
    int* idst = a.idx[1 - buf];
    const int rho = a.rho;
    const int start = ji[JI_START], NA = ji[JI_NA], first = ji[JI_FIRST];
    const Lanes<LP, D> L;
    double fa[D], fb[D];
    load_center(a.fa + job * rho, rho, L.d0, fa);
    load_center(a.fb + job * rho, rho, L.d0, fb);
    // members of the first child in the earlier blocks of this job
    int acc = 0;
    for (int q = threadIdx.x; q < rank; q += KT) acc += a.blkA[first + q];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (L.lane == 0) red[L.wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < KWAVES; ++q) t += red[q];
        s_offA = start + t;
        s_offB = start + NA + ((s - start) - t);
    }
    __syncthreads();
    int offA = s_offA, offB = s_offB;
    // each step visits KWAVES * PPW consecutive points: wave w takes the w-th
    // run of PPW, lane group pw its pw-th point
    for (int base = 0; base < cnt; base += KWAVES * L.PPW) {
        const int p = base + L.wave * L.PPW + L.pw;
        const bool valid = p < cnt;
        double x[D];
        load_dims<LP, D>(src, valid ? s + p : s, L.d0, x);
        const bool A = to_first<LP, D>(x, fa, fb, rho, L.d0);
        const bool lead = valid && L.sub == 0;
        const unsigned long long ma = __ballot(lead && A);
        const unsigned long long mb = __ballot(lead && !A);
        const int rl = L.lane & ~(LP - 1);  // the point's lead lane
        const unsigned long long bl = (rl == 0) ? 0ull : (~0ull >> (64 - rl));
        const int ra = __popcll(ma & bl), rb = __popcll(mb & bl);
        if (L.lane == 0) {
            s_wa[L.wave] = __popcll(ma);
            s_wb[L.wave] = __popcll(mb);
        }
        __syncthreads();
        int pa = 0, pb = 0, ta = 0, tb = 0;
        for (int q = 0; q < KWAVES; ++q) {
            if (q < L.wave) {
                pa += s_wa[q];
                pb += s_wb[q];
            }
            ta += s_wa[q];
            tb += s_wb[q];
        }
        if (valid) {
            const int to = A ? offA + pa + ra : offB + pb + rb;
            constexpr int PS = LP * D;
#pragma unroll
            for (int k = 0; k < D; ++k) dst[(long long)to * PS + L.d0 + k] = src[(long long)(s + p) * PS + L.d0 + k];
            if (L.sub == 0) idst[to] = isrc[s + p];
        }
        offA += ta;
        offB += tb;
        __syncthreads();
    }
}

// labels[pixel] = cluster index, for every member of every leaf.
__global__ __launch_bounds__(KT) void km_labels(KmArgs a, int* __restrict__ labels) {
    const int4 bt = a.btab[blockIdx.x];
    const int job = bjob(bt), s = bt.y, cnt = bt.z, lab = bt.w;
    const int* idx = a.idx[a.ji[job * JI_W + JI_BUF]];
    for (int p = threadIdx.x; p < cnt; p += KT) labels[idx[s + p]] = lab;
}

// ---------------------------------------------------------------------------
// finalize kernels: one block per job

__global__ __launch_bounds__(FT) void fin_stats(KmArgs a) {
    __shared__ double tmp[FT];
    __shared__ double res[3 * FHD_MAX_RHO];
    const int job = blockIdx.x, rho = a.rho;
    const int* ji = a.ji + job * JI_W;
    reduce_records(a.part, ji[JI_FIRST], ji[JI_NBLK], a.pst, 0, 3 * rho,
                   [rho](int e) { return e < rho ? 0 : (e < 2 * rho ? 1 : 2); }, tmp, res);
    if (threadIdx.x < rho) a.jm[job * rho + threadIdx.x] = res[threadIdx.x] / (double)ji[JI_COUNT];
    if (threadIdx.x == 0) {
        int split = 0;
        for (int t = 0; t < rho; ++t) split |= res[2 * rho + t] != res[rho + t];
        a.jd[job * JD_W + JD_SPLA] = split;
    }
}

__global__ __launch_bounds__(FT) void fin_sse1(KmArgs a) {
    __shared__ double tmp[FT];
    __shared__ double res[1];
    const int job = blockIdx.x;
    const int* ji = a.ji + job * JI_W;
    reduce_records(a.part, ji[JI_FIRST], ji[JI_NBLK], a.pst, 0, 1, [](int) { return 0; }, tmp, res);
    if (threadIdx.x == 0) a.jd[job * JD_W + JD_SSEA] = res[0];
}

__global__ __launch_bounds__(KT) void fin_far(KmArgs a, int which) {
    __shared__ double rb[KWAVES];
    __shared__ int ri[KWAVES], rp[KWAVES];
    __shared__ int s_pos;
    const int job = blockIdx.x, rho = a.rho;
    const int* ji = a.ji + job * JI_W;
    const int first = ji[JI_FIRST], nblk = ji[JI_NBLK];
    double B = -1.0;
    int I = INT_MAX, P = -1;
    for (int b = threadIdx.x; b < nblk; b += KT) {
        const double* rec = a.part + first + b;
        const double rb0 = rec[0];
        const int bi = (int)rec[a.pst];
        if (rb0 > B || (rb0 == B && bi < I)) {
            B = rb0;
            I = bi;
            P = (int)rec[2 * a.pst];
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double ob = __shfl_xor(B, o, 64);
        const int oi = __shfl_xor(I, o, 64);
        const int op = __shfl_xor(P, o, 64);
        if (ob > B || (ob == B && oi < I)) {
            B = ob;
            I = oi;
            P = op;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        rb[wave] = B;
        ri[wave] = I;
        rp[wave] = P;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < KWAVES; ++q)
            if (rb[q] > B || (rb[q] == B && ri[q] < I)) {
                B = rb[q];
                I = ri[q];
                P = rp[q];
            }
        s_pos = P;
    }
    __syncthreads();
    const float* pts = a.pts[ji[JI_BUF]];
    if (threadIdx.x < rho)
        (which == 0 ? a.ca : a.cb)[job * rho + threadIdx.x] = pts[(long long)s_pos * a.ps + threadIdx.x];
    if (threadIdx.x < rho) {  // the seeds are the centers of assignment step 0
        double* c0 = a.cst + (long long)job * 2 * rho;
        c0[which * rho + threadIdx.x] = pts[(long long)s_pos * a.ps + threadIdx.x];
    }
}

// The decision on the last assignment step T - 1 of the jobs still running:
// every outcome stops the job.
__global__ __launch_bounds__(FT) void fin_lloyd(KmArgs a, int T) {
    __shared__ double tmp[FT];
    __shared__ double res[2 * FHD_MAX_RHO + 2];
    __shared__ int s_act;
    const int job = blockIdx.x, rho = a.rho;
    if (a.jstop[(long long)((T - 1) & 1) * a.mj + job]) return;
    const int* ji = a.ji + job * JI_W;
    reduce_records((T - 1) & 1 ? a.part2 : a.part, ji[JI_FIRST], ji[JI_NBLK], a.pst, 0, 2 * rho + 2,
                   [](int) { return 0; }, tmp, res);
    const double* c = a.cst + ((long long)((T - 1) % 3) * a.mj + job) * 2 * rho;
    if (threadIdx.x == 0) s_act = lloyd_act(res, c, rho, T - 1);
    __syncthreads();
    lloyd_final(a, job, s_act, T - 1, res);
}

__global__ __launch_bounds__(FT) void fin_split(KmArgs a) {
    __shared__ double tmp[FT];
    __shared__ double res[4 + 4 * FHD_MAX_RHO];
    const int job = blockIdx.x, rho = a.rho;
    int* ji = a.ji + job * JI_W;
    reduce_records(
        a.part, ji[JI_FIRST], ji[JI_NBLK], a.pst, 0, 4 + 4 * rho,
        [rho](int e) {
            if (e < 4) return 0;
            const int q = (e - 4) / rho;
            return (q == 0 || q == 2) ? 1 : 2;
        },
        tmp, res);
    if (threadIdx.x == 0) {
        int sa = 0, sb = 0;
        for (int t = 0; t < rho; ++t) {
            sa |= res[4 + rho + t] > res[4 + t];
            sb |= res[4 + 3 * rho + t] > res[4 + 2 * rho + t];
        }
        double* jd = a.jd + job * JD_W;
        jd[JD_SSEA] = sa ? res[0] : 0.0;  // a single-valued group has SSE exactly 0
        jd[JD_SSEB] = sb ? res[1] : 0.0;
        jd[JD_NA] = res[2];
        jd[JD_NB] = res[3];
        jd[JD_SPLA] = sa;
        jd[JD_SPLB] = sb;
        ji[JI_NA] = (int)res[2];
    }
}

// ---------------------------------------------------------------------------
// host side

struct Leaf {
    std::string heap;  // path from the root: "1", then '0' (first child) / '1'
    int img = 0;       // image (tree) of the batch
    int start = 0, count = 0, buf = 0;
    std::vector<double> mean;
    double sse = 0.0;
    bool splittable = false;
    bool has_split = false;
    std::vector<double> meanA, meanB;
    double sseA = 0.0, sseB = 0.0;
    int nA = 0, nB = 0;
    bool splA = false, splB = false;
};

// heap-id order: shallower first, then by path
bool heap_less(const std::string& a, const std::string& b) {
    if (a.size() != b.size()) return a.size() < b.size();
    return a < b;
}

int lanes_per_point(int rho) {
    int lp = 1;
    while (lp * DPL < rho) lp <<= 1;
    return lp;
}

// floats per packed point: LP * D of the layout launch_pass picks
int point_stride(int rho) {
    if (rho <= 3) return 3;
    if (rho <= 4) return 4;
    return lanes_per_point(rho) * DPL;
}

// points per block: 16 lane groups of four waves
long long chunk_points(int rho) { return (long long)KITERS * KWAVES * (64 / lanes_per_point(rho)); }

int max_jobs(int K, int images) { return images * std::max(2 * K, 4); }

long long max_blocks(long long N, int rho, int K, int images) {
    return N / chunk_points(rho) + 2LL * max_jobs(K, images) + 4;
}

int record_width(int rho) { return 4 * rho + 8; }

// The job tables exchanged with the host every round, in one layout shared
// by the pinned host staging and its device mirror, so that each direction
// is one copy: [btab | ji | jm | ca | cb | jd], each part 256-byte aligned.
struct TableLayout {
    size_t btab, ji, jm, ca, cb, jd, end;
    TableLayout(long long maxBlocks, int maxJobs, int rho) {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += align_up(bytes, 256);
            return o;
        };
        btab = take(sizeof(int4) * maxBlocks);
        ji = take(sizeof(int) * maxJobs * JI_W);
        jm = take(sizeof(double) * maxJobs * rho);
        ca = take(sizeof(double) * maxJobs * rho);
        cb = take(sizeof(double) * maxJobs * rho);
        jd = take(sizeof(double) * maxJobs * JD_W);
        end = off;
    }
};

struct KmBuffers {
    float* pts[2];
    int* idx[2];
    int4* btab;
    int* blkA;
    double* part;
    double* part2;
    double* cst;
    int* jstop;
    int* ji;
    double *jm, *ca, *cb, *fa, *fb, *jd;
    char* tables;  // device mirror of the host staging (TableLayout)
    long long maxBlocks;
    int maxJobs;
};

KmBuffers carve(Arena& ws, long long N, int rho, int K, int images) {
    KmBuffers b{};
    b.maxJobs = max_jobs(K, images);
    b.maxBlocks = max_blocks(N, rho, K, images);
    for (int q = 0; q < 2; ++q) {
        b.pts[q] = ws.take<float>((size_t)N * point_stride(rho) + 64);
        b.idx[q] = ws.take<int>((size_t)N);
    }
    const TableLayout L(b.maxBlocks, b.maxJobs, rho);
    b.tables = ws.take<char>(L.end);
    char* t = b.tables;
    b.btab = t ? reinterpret_cast<int4*>(t + L.btab) : nullptr;
    b.ji = t ? reinterpret_cast<int*>(t + L.ji) : nullptr;
    b.jm = t ? reinterpret_cast<double*>(t + L.jm) : nullptr;
    b.ca = t ? reinterpret_cast<double*>(t + L.ca) : nullptr;
    b.cb = t ? reinterpret_cast<double*>(t + L.cb) : nullptr;
    b.jd = t ? reinterpret_cast<double*>(t + L.jd) : nullptr;
    b.blkA = ws.take<int>((size_t)b.maxBlocks);
    b.part = ws.take<double>((size_t)b.maxBlocks * record_width(rho));  // entry-major, stride maxBlocks
    b.part2 = ws.take<double>((size_t)b.maxBlocks * record_width(rho));
    b.cst = ws.take<double>((size_t)3 * b.maxJobs * 2 * rho);
    b.jstop = ws.take<int>((size_t)2 * b.maxJobs);
    b.fa = ws.take<double>((size_t)b.maxJobs * rho);
    b.fb = ws.take<double>((size_t)b.maxJobs * rho);
    return b;
}

enum { P_STATS, P_SSE1, P_FAR, P_LLOYD, P_SPLIT, P_SCATTER };

template <int LP, int D>
void launch_lp(int which, dim3 g, hipStream_t s, const KmArgs& a, int arg) {
    switch (which) {
        case P_STATS: hipLaunchKernelGGL((km_stats<LP, D>), g, dim3(KT), 0, s, a); break;
        case P_SSE1: hipLaunchKernelGGL((km_sse1<LP, D>), g, dim3(KT), 0, s, a); break;
        case P_FAR: hipLaunchKernelGGL((km_far<LP, D>), g, dim3(KT), 0, s, a, arg); break;
        case P_LLOYD: hipLaunchKernelGGL((km_lloyd<LP, D>), g, dim3(KT), 0, s, a, arg); break;
        case P_SPLIT: hipLaunchKernelGGL((km_split<LP, D>), g, dim3(KT), 0, s, a); break;
        default: hipLaunchKernelGGL((km_scatter<LP, D>), g, dim3(KT), 0, s, a); break;
    }
}

// lane layout by guide dimension: one lane per point with three, four or
// eight dimensions, or LP lanes of eight dimensions each (point_stride agrees)
void launch_pass(int rho, int which, dim3 g, hipStream_t s, const KmArgs& a, int arg = 0) {
    if (rho <= 3) launch_lp<1, 3>(which, g, s, a, arg);
    else if (rho <= 4) launch_lp<1, 4>(which, g, s, a, arg);
    else if (rho <= 8) launch_lp<1, 8>(which, g, s, a, arg);
    else if (rho <= 16) launch_lp<2, 8>(which, g, s, a, arg);
    else if (rho <= 32) launch_lp<4, 8>(which, g, s, a, arg);
    else launch_lp<8, 8>(which, g, s, a, arg);
}

// Host staging layout (pinned): block table, job ints, job doubles.
struct Stage {
    int4* btab;
    int* ji;
    double* jm;
    double* ca;
    double* cb;
    double* jd;
};

}  // namespace

size_t kmeans_workspace(long long N, int rho, int K, int images) {
    Arena probe;  // counts only
    carve(probe, N, rho, K, images);
    return probe.used;
}

void kmeans_run(Ctx& c, Arena& ws, const float* guide, int rho, long long N, int K, int max_iter, int* labels,
                KmResult& out) {
    std::vector<KmResult> res;
    const long long off = 0;
    kmeans_run_batch(c, ws, guide, rho, 1, &off, &N, K, max_iter, labels, res);
    out = res[0];
}

void kmeans_run_batch(Ctx& c, Arena& ws, const float* guide, int rho, int images, const long long* px_offset,
                      const long long* px_count, int K, int max_iter, int* labels, std::vector<KmResult>& out) {
    FHD_REQUIRE(images >= 1, FHD_EINVAL, "no images");
    long long N = 0;
    for (int b = 0; b < images; ++b) {
        FHD_REQUIRE(px_count[b] >= 1 && px_offset[b] == N, FHD_EINVAL,
                    "internal: images must be packed back to back");
        N += px_count[b];
    }
    FHD_REQUIRE(N < (1LL << 31), FHD_EINVAL, "too many pixels for clustering");
    FHD_REQUIRE(rho >= 1 && rho <= FHD_MAX_RHO, FHD_EUNSUPPORTED, "guide dimension out of range");
    FHD_REQUIRE(K >= 1 && K <= FHD_MAX_K, FHD_EINVAL, "K out of range");
    FHD_REQUIRE(max_iter >= 1, FHD_EINVAL, "kmeans_max_iter must be >= 1");
    KmBuffers B = carve(ws, N, rho, K, images);
    const long long CH = chunk_points(rho);
    hipStream_t st = c.stream;

    const TableLayout TL(B.maxBlocks, B.maxJobs, rho);
    char* hs = static_cast<char*>(c.host_stage(0, TL.end));
    Stage H;
    H.btab = reinterpret_cast<int4*>(hs + TL.btab);
    H.ji = reinterpret_cast<int*>(hs + TL.ji);
    H.jm = reinterpret_cast<double*>(hs + TL.jm);
    H.ca = reinterpret_cast<double*>(hs + TL.ca);
    H.cb = reinterpret_cast<double*>(hs + TL.cb);
    H.jd = reinterpret_cast<double*>(hs + TL.jd);
    // one copy per direction: host -> device covers btab and ji (and jm),
    // device -> host covers jm, ca, cb and jd
    auto to_device = [&](size_t upto) {
        FHD_HIP(hipMemcpyAsync(B.tables, hs, upto, hipMemcpyHostToDevice, st));
    };
    auto to_host = [&](size_t from, size_t upto) {
        FHD_HIP(hipMemcpyAsync(hs + from, B.tables + from, upto - from, hipMemcpyDeviceToHost, st));
    };

    KmArgs a{};
    for (int q = 0; q < 2; ++q) {
        a.pts[q] = B.pts[q];
        a.idx[q] = B.idx[q];
    }
    a.btab = B.btab;
    a.blkA = B.blkA;
    a.part = B.part;
    a.ji = B.ji;
    a.jm = B.jm;
    a.ca = B.ca;
    a.cb = B.cb;
    a.part2 = B.part2;
    a.cst = B.cst;
    a.jstop = B.jstop;
    a.mj = B.maxJobs;
    a.fa = B.fa;
    a.fb = B.fb;
    a.jd = B.jd;
    a.rho = rho;
    a.pst = B.maxBlocks;
    a.ps = point_stride(rho);

    hipEvent_t t_begin = c.stage_begin();
    for (int b = 0; b < images; ++b)
        hipLaunchKernelGGL(km_pack, dim3((unsigned)((px_count[b] + KT - 1) / KT)), dim3(KT), 0, st,
                           guide + (size_t)rho * px_offset[b], rho, a.ps, px_count[b], px_offset[b], B.pts[0],
                           B.idx[0]);
    FHD_HIP(hipGetLastError());

    // Upload jobs (ranges of leaves) and their block table; returns #blocks.
    // The block table's last field is the block's rank within its job, or
    // the job's label when `label` is given.
    auto upload = [&](const std::vector<Leaf*>& jobs, bool with_mean, const std::vector<int>* label) -> int {
        int nb = 0;
        for (size_t j = 0; j < jobs.size(); ++j) {
            const Leaf& L = *jobs[j];
            const int nblk = (int)((L.count + CH - 1) / CH);
            int* ji = H.ji + j * JI_W;
            std::memset(ji, 0, sizeof(int) * JI_W);
            ji[JI_START] = L.start;
            ji[JI_COUNT] = L.count;
            ji[JI_BUF] = L.buf;
            ji[JI_FIRST] = nb;
            ji[JI_NBLK] = nblk;
            for (int q = 0; q < nblk; ++q) {
                const int s0 = L.start + (int)(q * CH);
                const int cnt = (int)std::min<long long>(CH, L.count - q * CH);
                H.btab[nb++] = make_int4((int)j | (L.buf << 30), s0, cnt, label ? (*label)[j] : q);
            }
            if (with_mean)
                for (int t = 0; t < rho; ++t) H.jm[j * rho + t] = L.mean[t];
        }
        FHD_REQUIRE(nb <= B.maxBlocks, FHD_EINVAL, "internal: block table overflow");
        to_device(with_mean ? TL.jm + sizeof(double) * rho * jobs.size() : TL.ji + sizeof(int) * JI_W * jobs.size());
        return nb;
    };

    // ---- roots: centroid, SSE, splittable (all images in one pass)
    std::vector<Leaf> store;
    store.reserve((size_t)images * (4 * (size_t)K + 4));
    std::vector<std::vector<Leaf*>> leaves(images);
    {
        std::vector<Leaf*> roots;
        for (int b = 0; b < images; ++b) {
            store.emplace_back();
            Leaf* r = &store.back();
            r->heap = "1";
            r->img = b;
            r->start = (int)px_offset[b];
            r->count = (int)px_count[b];
            r->buf = 0;
            roots.push_back(r);
            leaves[b].push_back(r);
        }
        const int nb = upload(roots, false, nullptr);
        const dim3 gj((unsigned)images);
        launch_pass(rho, P_STATS, dim3(nb), st, a);
        hipLaunchKernelGGL(fin_stats, gj, dim3(FT), 0, st, a);
        launch_pass(rho, P_SSE1, dim3(nb), st, a);
        hipLaunchKernelGGL(fin_sse1, gj, dim3(FT), 0, st, a);
        FHD_HIP(hipGetLastError());
        to_host(TL.jm, TL.jd + sizeof(double) * JD_W * images);
        FHD_HIP(hipStreamSynchronize(st));
        for (int b = 0; b < images; ++b) {
            Leaf* r = roots[b];
            r->mean.assign(H.jm + (size_t)b * rho, H.jm + (size_t)(b + 1) * rho);
            r->splittable = H.jd[(size_t)b * JD_W + JD_SPLA] != 0.0;
            r->sse = r->splittable ? H.jd[(size_t)b * JD_W + JD_SSEA] : 0.0;
        }
    }

    std::vector<int> rounds(images, 0), splits(images, 0);
    auto rank_less = [](const Leaf* x, const Leaf* y) {
        if (x->sse != y->sse) return x->sse > y->sse;
        return heap_less(x->heap, y->heap);
    };
    auto open_leaf = [](const Leaf* L) { return L->splittable && L->sse > 0.0; };
    for (;;) {
        // per image: the leaves its greedy rule can still pick, the top
        // (K - #leaves) open ones; their missing splits are this round's jobs
        std::vector<Leaf*> jobs;
        bool active = false;
        for (int b = 0; b < images; ++b) {
            if ((int)leaves[b].size() >= K) continue;
            std::vector<Leaf*> cand;
            for (Leaf* L : leaves[b])
                if (open_leaf(L)) cand.push_back(L);
            if (cand.empty()) continue;
            active = true;
            std::sort(cand.begin(), cand.end(), rank_less);
            const size_t budget = (size_t)K - leaves[b].size();
            if (cand.size() > budget) cand.resize(budget);
            bool mine = false;
            for (Leaf* L : cand)
                if (!L->has_split) {
                    jobs.push_back(L);
                    mine = true;
                }
            if (mine) ++rounds[b];
        }
        if (!active) break;
        if (!jobs.empty()) {
            FHD_REQUIRE((int)jobs.size() <= B.maxJobs, FHD_EINVAL, "internal: too many jobs");
            const int nb = upload(jobs, true, nullptr);
            const dim3 g(nb), gj((unsigned)jobs.size());
            launch_pass(rho, P_FAR, g, st, a, 0);
            hipLaunchKernelGGL(fin_far, gj, dim3(KT), 0, st, a, 0);
            launch_pass(rho, P_FAR, g, st, a, 1);
            hipLaunchKernelGGL(fin_far, gj, dim3(KT), 0, st, a, 1);
            hipEvent_t tl = c.stage_begin();
            for (int it = 0; it < max_iter; ++it) launch_pass(rho, P_LLOYD, g, st, a, it);
            c.stage_end(FHD_STAGE_LLOYD, tl, max_iter);
            hipLaunchKernelGGL(fin_lloyd, gj, dim3(FT), 0, st, a, max_iter);
            launch_pass(rho, P_SPLIT, g, st, a);
            hipLaunchKernelGGL(fin_split, gj, dim3(FT), 0, st, a);
            launch_pass(rho, P_SCATTER, g, st, a);
            FHD_HIP(hipGetLastError());
            const size_t J = jobs.size();
            to_host(TL.ca, TL.jd + sizeof(double) * JD_W * J);
            FHD_HIP(hipStreamSynchronize(st));
            for (size_t j = 0; j < J; ++j) {
                Leaf& L = *jobs[j];
                const double* jd = H.jd + j * JD_W;
                L.has_split = true;
                L.meanA.assign(H.ca + j * rho, H.ca + (j + 1) * rho);
                L.meanB.assign(H.cb + j * rho, H.cb + (j + 1) * rho);
                L.sseA = jd[JD_SSEA];
                L.sseB = jd[JD_SSEB];
                L.nA = (int)jd[JD_NA];
                L.nB = (int)jd[JD_NB];
                L.splA = jd[JD_SPLA] != 0.0;
                L.splB = jd[JD_SPLB] != 0.0;
                if (c.timing) c.units[FHD_STAGE_LLOYD] += (long long)jd[JD_STEPS] * L.count;
                FHD_REQUIRE(L.nA > 0 && L.nB > 0 && L.nA + L.nB == L.count, FHD_ENUMERIC,
                            "internal: degenerate 2-means split");
                ++splits[L.img];
            }
        }
        // commit greedily, per image, while its best leaf's split is known
        for (int b = 0; b < images; ++b) {
            std::vector<Leaf*>& lv = leaves[b];
            while ((int)lv.size() < K) {
                Leaf* best = nullptr;
                for (Leaf* L : lv)
                    if (open_leaf(L) && (best == nullptr || rank_less(L, best))) best = L;
                if (best == nullptr || !best->has_split) break;
                store.emplace_back();
                Leaf* A = &store.back();
                store.emplace_back();
                Leaf* Bc = &store.back();
                A->heap = best->heap + "0";
                A->img = b;
                A->start = best->start;
                A->count = best->nA;
                A->buf = 1 - best->buf;
                A->mean = best->meanA;
                A->sse = best->sseA;
                A->splittable = best->splA;
                Bc->heap = best->heap + "1";
                Bc->img = b;
                Bc->start = best->start + best->nA;
                Bc->count = best->nB;
                Bc->buf = 1 - best->buf;
                Bc->mean = best->meanB;
                Bc->sse = best->sseB;
                Bc->splittable = best->splB;
                lv.erase(std::find(lv.begin(), lv.end(), best));
                lv.push_back(A);
                lv.push_back(Bc);
            }
        }
    }

    out.assign(images, KmResult{});
    std::vector<Leaf*> all;
    std::vector<int> lab;
    for (int b = 0; b < images; ++b) {
        std::vector<Leaf*>& lv = leaves[b];
        std::sort(lv.begin(), lv.end(), [](const Leaf* x, const Leaf* y) { return heap_less(x->heap, y->heap); });
        KmResult& r = out[b];
        r.K_eff = (int)lv.size();
        r.rounds = rounds[b];
        r.splits = splits[b];
        r.E_K = 0.0;
        r.centers.assign((size_t)r.K_eff * rho, 0.0);
        for (int k = 0; k < r.K_eff; ++k) {
            r.E_K += lv[k]->sse;
            for (int t = 0; t < rho; ++t) r.centers[(size_t)k * rho + t] = lv[k]->mean[t];
            all.push_back(lv[k]);
            lab.push_back(k);
        }
    }
    if (labels != nullptr) {
        FHD_REQUIRE((int)all.size() <= B.maxJobs, FHD_EINVAL, "internal: too many leaves");
        const int nb = upload(all, false, &lab);
        hipLaunchKernelGGL(km_labels, dim3(nb), dim3(KT), 0, st, a, labels);
        FHD_HIP(hipGetLastError());
    }
    c.stage_end(FHD_STAGE_CLUSTER, t_begin);
    c.stage_done(0);
}

}  // namespace fhd
