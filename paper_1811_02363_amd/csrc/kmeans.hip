// Bisecting K-means of the range space (Algorithm 1, step 1; Sec. II-C) on
// the GPU.
//
// Design: the guide vectors are packed point-major (AoS) together with their
// pixel index, and every cluster is kept as a contiguous range of that array
// (two ping-pong copies; a split stably partitions its range into the other
// copy).  Splits are computed in batched rounds: each round computes, for all
// leaves that the greedy largest-SSE rule may still pick, the 2-means split
// (seeds, Lloyd steps, children's SSE, partition) with one launch per pass for
// all of them.  The host then commits splits greedily and plans the next
// round; this is the only host synchronisation, once per round.
//
// Arithmetic: distances and centroid sums in FP64, reduced in a fixed order
// (per-lane sequential, fixed shuffle tree, then blocks in index order), so a
// run is deterministic.  No floating-point atomics.  A block's lanes are laid
// out dimension-parallel: LP = next power of two >= rho lanes per point.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>

#include "fhd_internal.h"

namespace fhd {
namespace {

constexpr int KT = 256;          // threads per block
constexpr int KWAVES = KT / 64;  // waves per block
constexpr int KITERS = 32;       // point groups per block and pass

// per-job integer state
enum { JI_START, JI_COUNT, JI_BUF, JI_CONV, JI_PARITY, JI_ITERS, JI_FIRST, JI_NBLK, JI_NA, JI_W = 12 };
// per-job FP64 results
enum { JD_MAXD, JD_SSEA, JD_SSEB, JD_NA, JD_NB, JD_SPLA, JD_SPLB, JD_W = 8 };

struct KmArgs {
    float* pts[2];
    int* idx[2];
    unsigned char* side[2];
    const int4* btab;  // per block: job, first point, point count, rank within job (or label)
    int* blkA;         // per block: members assigned to the first child
    double* part;      // per block partials, pw doubles each
    int* ji;           // per job ints, JI_W each
    double* jm;        // per job centroid (rho)
    double* ca;        // per job first seed / child centroid (rho)
    double* cb;        // per job second seed / child centroid (rho)
    double* jd;        // per job results, JD_W each
    unsigned* done;    // per job finished-block counters (zero between passes)
    int rho;
    int pw;
};

template <int LP>
__device__ inline double sum_over_point(double v) {
#pragma unroll
    for (int o = 1; o < LP; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reduce `v` over the lanes of the block that hold the same dimension
// (lane % LP); thread t < LP receives the total for dimension t.  OP: 0 sum,
// 1 min, 2 max.  Fixed order: shuffle tree, then waves 0..3.
template <int LP, int OP>
__device__ inline double block_reduce_dims(double v, double (*red)[64]) {
#pragma unroll
    for (int o = LP; o < 64; o <<= 1) {
        double w = __shfl_xor(v, o, 64);
        v = OP == 0 ? v + w : (OP == 1 ? fmin(v, w) : fmax(v, w));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane < LP) red[wave][lane] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < LP) {
        r = red[0][threadIdx.x];
        for (int q = 1; q < KWAVES; ++q) {
            double w = red[q][threadIdx.x];
            r = OP == 0 ? r + w : (OP == 1 ? fmin(r, w) : fmax(r, w));
        }
    }
    return r;
}

// Sum of `v` over every lane of the block; valid in thread 0.
__device__ inline double block_sum_all(double v, double (*red)[64]) {
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

// True in every thread of the block that is the last of its job to finish
// this pass.  Partials written before the call are visible to that block.
__device__ inline bool last_block(unsigned* done, int job, int nblk) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = __hip_atomic_fetch_add(&done[job], 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (unsigned)(nblk - 1)) ? 1 : 0;
    }
    __syncthreads();
    const bool last = s_last != 0;
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) done[job] = 0u;
    }
    return last;
}

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(KT) void km_pack(const float* __restrict__ guide, int rho,
                                              long long N, float* __restrict__ pts,
                                              int* __restrict__ idx) {
    const long long i = (long long)blockIdx.x * KT + threadIdx.x;
    if (i >= N) return;
    for (int d = 0; d < rho; ++d) pts[i * rho + d] = guide[(long long)d * N + i];
    idx[i] = (int)i;
}

// Centroid (sum / count) and per-dimension min/max of each job's members.
template <int LP>
__global__ __launch_bounds__(KT) void km_stats(KmArgs a) {
    __shared__ double red[KWAVES][64];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bt.x, s = bt.y, cnt = bt.z;
    const int* ji = a.ji + job * JI_W;
    const float* pts = a.pts[ji[JI_BUF]];
    const int rho = a.rho;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = lane & (LP - 1), pw = lane / LP;
    constexpr int PPW = 64 / LP;
    double sum = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int base = 0; base < cnt; base += KWAVES * PPW) {
        const int p = base + wave * PPW + pw;
        if (p < cnt && d < rho) {
            const double x = pts[(long long)(s + p) * rho + d];
            sum += x;
            mn = fmin(mn, x);
            mx = fmax(mx, x);
        }
    }
    double* part = a.part + (long long)blockIdx.x * a.pw;
    const double tsum = block_reduce_dims<LP, 0>(sum, red);
    const double tmn = block_reduce_dims<LP, 1>(mn, red);
    const double tmx = block_reduce_dims<LP, 2>(mx, red);
    if (threadIdx.x < rho) {
        part[threadIdx.x] = tsum;
        part[rho + threadIdx.x] = tmn;
        part[2 * rho + threadIdx.x] = tmx;
    }
    if (!last_block(a.done, job, ji[JI_NBLK])) return;
    __shared__ int s_split;
    if (threadIdx.x == 0) s_split = 0;
    __syncthreads();
    if (threadIdx.x < rho) {
        const int t = threadIdx.x;
        double S = 0.0, lo = INFINITY, hi = -INFINITY;
        for (int b = ji[JI_FIRST]; b < ji[JI_FIRST] + ji[JI_NBLK]; ++b) {
            const double* pb = a.part + (long long)b * a.pw;
            S += pb[t];
            lo = fmin(lo, pb[rho + t]);
            hi = fmax(hi, pb[2 * rho + t]);
        }
        a.jm[job * rho + t] = S / (double)ji[JI_COUNT];
        if (hi != lo) atomicOr(&s_split, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) a.jd[job * JD_W + JD_SPLA] = (double)s_split;
}

// Seed search: the member farthest from the centroid (which == 0, stored in
// ca) or from the first seed (which == 1, stored in cb); ties -> lowest pixel
// index.
template <int LP>
__global__ __launch_bounds__(KT) void km_far(KmArgs a, int which) {
    __shared__ double rb[KWAVES];
    __shared__ int ri[KWAVES], rp[KWAVES];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bt.x, s = bt.y, cnt = bt.z;
    const int* ji = a.ji + job * JI_W;
    const float* pts = a.pts[ji[JI_BUF]];
    const int* idx = a.idx[ji[JI_BUF]];
    const int rho = a.rho;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = lane & (LP - 1), pw = lane / LP;
    constexpr int PPW = 64 / LP;
    const double* ref = (which == 0 ? a.jm : a.ca) + job * rho;
    const double r = d < rho ? ref[d] : 0.0;
    double best = -1.0;
    int bidx = INT_MAX, bpos = -1;
    for (int base = 0; base < cnt; base += KWAVES * PPW) {
        const int p = base + wave * PPW + pw;
        const bool valid = p < cnt;
        double t = 0.0;
        if (valid && d < rho) {
            const double x = pts[(long long)(s + p) * rho + d];
            t = (x - r) * (x - r);
        }
        t = sum_over_point<LP>(t);
        if (valid) {
            const int pi = idx[s + p];
            if (t > best || (t == best && pi < bidx)) {
                best = t;
                bidx = pi;
                bpos = s + p;
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
    if (lane == 0) {
        rb[wave] = best;
        ri[wave] = bidx;
        rp[wave] = bpos;
    }
    __syncthreads();
    double* part = a.part + (long long)blockIdx.x * a.pw;
    if (threadIdx.x == 0) {
        for (int q = 1; q < KWAVES; ++q)
            if (rb[q] > best || (rb[q] == best && ri[q] < bidx)) {
                best = rb[q];
                bidx = ri[q];
                bpos = rp[q];
            }
        part[0] = best;
        part[1] = (double)bidx;
        part[2] = (double)bpos;
    }
    if (!last_block(a.done, job, ji[JI_NBLK])) return;
    __shared__ int s_pos;
    if (threadIdx.x == 0) {
        double B = -1.0;
        int I = INT_MAX, P = -1;
        for (int b = ji[JI_FIRST]; b < ji[JI_FIRST] + ji[JI_NBLK]; ++b) {
            const double* pb = a.part + (long long)b * a.pw;
            const int bi = (int)pb[1];
            if (pb[0] > B || (pb[0] == B && bi < I)) {
                B = pb[0];
                I = bi;
                P = (int)pb[2];
            }
        }
        s_pos = P;
        if (which == 0) a.jd[job * JD_W + JD_MAXD] = B;
    }
    __syncthreads();
    if (threadIdx.x < rho) {
        double* dst = (which == 0 ? a.ca : a.cb) + job * rho;
        dst[threadIdx.x] = pts[(long long)s_pos * rho + threadIdx.x];
    }
}

// One 2-means assignment step: x joins the first child iff
// |x - c_a|^2 <= |x - c_b|^2; then the children's centroids are updated.  The
// labels of step `it` go to side[it & 1]; the previous step's labels are in
// side[(it + 1) & 1].
template <int LP>
__global__ __launch_bounds__(KT) void km_lloyd(KmArgs a, int it, int T) {
    __shared__ double red[KWAVES][64];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bt.x, s = bt.y, cnt = bt.z;
    int* ji = a.ji + job * JI_W;
    if (ji[JI_CONV]) return;
    const float* pts = a.pts[ji[JI_BUF]];
    const int rho = a.rho;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = lane & (LP - 1), pw = lane / LP;
    constexpr int PPW = 64 / LP;
    const double ca = d < rho ? a.ca[job * rho + d] : 0.0;
    const double cb = d < rho ? a.cb[job * rho + d] : 0.0;
    unsigned char* snew = a.side[it & 1];
    const unsigned char* sold = a.side[(it + 1) & 1];
    double sa = 0.0, sb = 0.0, na = 0.0, nb = 0.0, ch = 0.0;
    for (int base = 0; base < cnt; base += KWAVES * PPW) {
        const int p = base + wave * PPW + pw;
        const bool valid = p < cnt;
        double x = 0.0, ta = 0.0, tb = 0.0;
        if (valid && d < rho) {
            x = pts[(long long)(s + p) * rho + d];
            ta = (x - ca) * (x - ca);
            tb = (x - cb) * (x - cb);
        }
        ta = sum_over_point<LP>(ta);
        tb = sum_over_point<LP>(tb);
        if (valid) {
            const bool toA = ta <= tb;
            if (toA) sa += x; else sb += x;
            if (d == 0) {
                const unsigned char ns = toA ? 0 : 1;
                if (toA) na += 1.0; else nb += 1.0;
                if (it > 0 && sold[s + p] != ns) ch += 1.0;
                snew[s + p] = ns;
            }
        }
    }
    const double tsa = block_reduce_dims<LP, 0>(sa, red);
    const double tsb = block_reduce_dims<LP, 0>(sb, red);
    const double tna = block_sum_all(na, red);
    const double tnb = block_sum_all(nb, red);
    const double tch = block_sum_all(ch, red);
    double* part = a.part + (long long)blockIdx.x * a.pw;
    if (threadIdx.x < rho) {
        part[threadIdx.x] = tsa;
        part[rho + threadIdx.x] = tsb;
    }
    if (threadIdx.x == 0) {
        part[2 * rho] = tna;
        part[2 * rho + 1] = tnb;
        part[2 * rho + 2] = tch;
    }
    if (!last_block(a.done, job, ji[JI_NBLK])) return;
    __shared__ double s_na, s_nb;
    __shared__ int s_update;
    const int first = ji[JI_FIRST], nblk = ji[JI_NBLK];
    if (threadIdx.x == 0) {
        double NA = 0.0, NB = 0.0, CH = 0.0;
        for (int b = first; b < first + nblk; ++b) {
            const double* pb = a.part + (long long)b * a.pw;
            NA += pb[2 * rho];
            NB += pb[2 * rho + 1];
            CH += pb[2 * rho + 2];
        }
        int update = 0;
        if (it > 0 && CH == 0.0) {
            ji[JI_CONV] = 1;  // no label changed: centroids already match
            ji[JI_PARITY] = it & 1;
        } else if (NA == 0.0 || NB == 0.0) {
            ji[JI_CONV] = 1;  // a child would be empty: keep the previous step
            ji[JI_PARITY] = (it + 1) & 1;
        } else {
            update = 1;
            ji[JI_PARITY] = it & 1;
            ji[JI_ITERS] = it + 1;
            if (it == T - 1) ji[JI_CONV] = 1;
        }
        s_na = NA;
        s_nb = NB;
        s_update = update;
    }
    __syncthreads();
    if (s_update && threadIdx.x < rho) {
        const int t = threadIdx.x;
        double SA = 0.0, SB = 0.0;
        for (int b = first; b < first + nblk; ++b) {
            const double* pb = a.part + (long long)b * a.pw;
            SA += pb[t];
            SB += pb[rho + t];
        }
        a.ca[job * rho + t] = SA / s_na;
        a.cb[job * rho + t] = SB / s_nb;
    }
}

// SSE, member counts and per-dimension min/max of the two children (split
// mode: labels side[parity], centroids ca/cb) or of the whole job (single
// mode: every member in the first group, centroid jm).
template <int LP>
__global__ __launch_bounds__(KT) void km_sse(KmArgs a, int single) {
    __shared__ double red[KWAVES][64];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bt.x, s = bt.y, cnt = bt.z;
    int* ji = a.ji + job * JI_W;
    const float* pts = a.pts[ji[JI_BUF]];
    const int rho = a.rho;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = lane & (LP - 1), pw = lane / LP;
    constexpr int PPW = 64 / LP;
    const double ca = d < rho ? (single ? a.jm : a.ca)[job * rho + d] : 0.0;
    const double cb = (d < rho && !single) ? a.cb[job * rho + d] : 0.0;
    const unsigned char* sd = a.side[ji[JI_PARITY]];
    double ea = 0.0, eb = 0.0, na = 0.0, nb = 0.0;
    double mna = INFINITY, mxa = -INFINITY, mnb = INFINITY, mxb = -INFINITY;
    for (int base = 0; base < cnt; base += KWAVES * PPW) {
        const int p = base + wave * PPW + pw;
        if (p >= cnt) continue;
        const bool inB = single ? false : (sd[s + p] != 0);
        if (d < rho) {
            const double x = pts[(long long)(s + p) * rho + d];
            if (inB) {
                eb += (x - cb) * (x - cb);
                mnb = fmin(mnb, x);
                mxb = fmax(mxb, x);
            } else {
                ea += (x - ca) * (x - ca);
                mna = fmin(mna, x);
                mxa = fmax(mxa, x);
            }
        }
        if (d == 0) {
            if (inB) nb += 1.0; else na += 1.0;
        }
    }
    const double tea = block_sum_all(ea, red);
    const double teb = block_sum_all(eb, red);
    const double tna = block_sum_all(na, red);
    const double tnb = block_sum_all(nb, red);
    const double t0 = block_reduce_dims<LP, 1>(mna, red);
    const double t1 = block_reduce_dims<LP, 2>(mxa, red);
    const double t2 = block_reduce_dims<LP, 1>(mnb, red);
    const double t3 = block_reduce_dims<LP, 2>(mxb, red);
    double* part = a.part + (long long)blockIdx.x * a.pw;
    if (threadIdx.x == 0) {
        part[0] = tea;
        part[1] = teb;
        part[2] = tna;
        part[3] = tnb;
        a.blkA[blockIdx.x] = (int)tna;
    }
    if (threadIdx.x < rho) {
        part[4 + threadIdx.x] = t0;
        part[4 + rho + threadIdx.x] = t1;
        part[4 + 2 * rho + threadIdx.x] = t2;
        part[4 + 3 * rho + threadIdx.x] = t3;
    }
    if (!last_block(a.done, job, ji[JI_NBLK])) return;
    __shared__ int s_sa, s_sb;
    const int first = ji[JI_FIRST], nblk = ji[JI_NBLK];
    if (threadIdx.x == 0) {
        s_sa = 0;
        s_sb = 0;
    }
    __syncthreads();
    if (threadIdx.x < rho) {
        const int t = threadIdx.x;
        double lo_a = INFINITY, hi_a = -INFINITY, lo_b = INFINITY, hi_b = -INFINITY;
        for (int b = first; b < first + nblk; ++b) {
            const double* pb = a.part + (long long)b * a.pw;
            lo_a = fmin(lo_a, pb[4 + t]);
            hi_a = fmax(hi_a, pb[4 + rho + t]);
            lo_b = fmin(lo_b, pb[4 + 2 * rho + t]);
            hi_b = fmax(hi_b, pb[4 + 3 * rho + t]);
        }
        if (hi_a > lo_a) atomicOr(&s_sa, 1);
        if (hi_b > lo_b) atomicOr(&s_sb, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double EA = 0.0, EB = 0.0, NA = 0.0, NB = 0.0;
        for (int b = first; b < first + nblk; ++b) {
            const double* pb = a.part + (long long)b * a.pw;
            EA += pb[0];
            EB += pb[1];
            NA += pb[2];
            NB += pb[3];
        }
        double* jd = a.jd + job * JD_W;
        jd[JD_SSEA] = s_sa ? EA : 0.0;  // a single-valued group has SSE exactly 0
        jd[JD_SSEB] = s_sb ? EB : 0.0;
        jd[JD_NA] = NA;
        jd[JD_NB] = NB;
        jd[JD_SPLA] = s_sa;
        jd[JD_SPLB] = s_sb;
        ji[JI_NA] = (int)NA;
    }
}

// Stable partition of each job's range by the final labels into the other
// copy: first-child members first, both groups in their original order.
__global__ __launch_bounds__(KT) void km_scatter(KmArgs a) {
    __shared__ int red[KWAVES];
    __shared__ int s_offA, s_offB, s_wa[KWAVES], s_wb[KWAVES];
    const int4 bt = a.btab[blockIdx.x];
    const int job = bt.x, s = bt.y, cnt = bt.z, rank = bt.w;
    const int* ji = a.ji + job * JI_W;
    const int buf = ji[JI_BUF];
    const float* src = a.pts[buf];
    const int* isrc = a.idx[buf];
    float* dst = a.pts[1 - buf];
    int* idst = a.idx[1 - buf];
    const int rho = a.rho;
    const int start = ji[JI_START], NA = ji[JI_NA], first = ji[JI_FIRST];
    const unsigned char* sd = a.side[ji[JI_PARITY]];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // members of the first child in the earlier blocks of this job
    int acc = 0;
    for (int q = threadIdx.x; q < rank; q += KT) acc += a.blkA[first + q];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < KWAVES; ++q) t += red[q];
        s_offA = start + t;
        s_offB = start + NA + ((s - start) - t);
    }
    __syncthreads();
    int offA = s_offA, offB = s_offB;
    for (int base = 0; base < cnt; base += KT) {
        const int p = base + threadIdx.x;
        const bool valid = p < cnt;
        const bool inA = valid && sd[s + p] == 0;
        const bool inB = valid && !inA;
        const unsigned long long ma = __ballot(inA);
        const unsigned long long mb = __ballot(inB);
        const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int ra = __popcll(ma & below), rb = __popcll(mb & below);
        if (lane == 0) {
            s_wa[wave] = __popcll(ma);
            s_wb[wave] = __popcll(mb);
        }
        __syncthreads();
        int pa = 0, pb = 0, ta = 0, tb = 0;
        for (int q = 0; q < KWAVES; ++q) {
            if (q < wave) {
                pa += s_wa[q];
                pb += s_wb[q];
            }
            ta += s_wa[q];
            tb += s_wb[q];
        }
        if (valid) {
            const int to = inA ? offA + pa + ra : offB + pb + rb;
            for (int dd = 0; dd < rho; ++dd)
                dst[(long long)to * rho + dd] = src[(long long)(s + p) * rho + dd];
            idst[to] = isrc[s + p];
        }
        offA += ta;
        offB += tb;
        __syncthreads();
    }
}

// labels[pixel] = cluster index, for every member of every leaf.
__global__ __launch_bounds__(KT) void km_labels(KmArgs a, int* __restrict__ labels) {
    const int4 bt = a.btab[blockIdx.x];
    const int job = bt.x, s = bt.y, cnt = bt.z, lab = bt.w;
    const int* idx = a.idx[a.ji[job * JI_W + JI_BUF]];
    for (int p = threadIdx.x; p < cnt; p += KT) labels[idx[s + p]] = lab;
}

// ---------------------------------------------------------------------------
// host side

struct Leaf {
    std::string heap;  // path from the root: "1", then '0' (first child) / '1'
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
    while (lp < rho) lp <<= 1;
    return lp;
}

struct KmBuffers {
    float* pts[2];
    int* idx[2];
    unsigned char* side[2];
    int4* btab;
    int* blkA;
    double* part;
    int* ji;
    double *jm, *ca, *cb, *jd;
    unsigned* done;
    long long maxBlocks;
    int maxJobs;
};

long long chunk_points(int rho) { return (long long)KITERS * KWAVES * (64 / lanes_per_point(rho)); }

long long max_blocks(long long N, int rho, int K) { return N / chunk_points(rho) + 2LL * K + 4; }

KmBuffers carve(Arena& ws, long long N, int rho, int K) {
    KmBuffers b{};
    b.maxJobs = std::max(2 * K, 4);
    b.maxBlocks = max_blocks(N, rho, K);
    for (int q = 0; q < 2; ++q) {
        b.pts[q] = ws.take<float>((size_t)N * rho);
        b.idx[q] = ws.take<int>((size_t)N);
        b.side[q] = ws.take<unsigned char>((size_t)N);
    }
    b.btab = ws.take<int4>((size_t)b.maxBlocks);
    b.blkA = ws.take<int>((size_t)b.maxBlocks);
    b.part = ws.take<double>((size_t)b.maxBlocks * (4 * rho + 8));
    b.ji = ws.take<int>((size_t)b.maxJobs * JI_W);
    b.jm = ws.take<double>((size_t)b.maxJobs * rho);
    b.ca = ws.take<double>((size_t)b.maxJobs * rho);
    b.cb = ws.take<double>((size_t)b.maxJobs * rho);
    b.jd = ws.take<double>((size_t)b.maxJobs * JD_W);
    b.done = ws.take<unsigned>((size_t)b.maxJobs);
    return b;
}

template <int LP>
struct Passes {
    static void stats(dim3 g, hipStream_t s, const KmArgs& a) {
        hipLaunchKernelGGL(km_stats<LP>, g, dim3(KT), 0, s, a);
    }
    static void far(dim3 g, hipStream_t s, const KmArgs& a, int which) {
        hipLaunchKernelGGL(km_far<LP>, g, dim3(KT), 0, s, a, which);
    }
    static void lloyd(dim3 g, hipStream_t s, const KmArgs& a, int it, int T) {
        hipLaunchKernelGGL(km_lloyd<LP>, g, dim3(KT), 0, s, a, it, T);
    }
    static void sse(dim3 g, hipStream_t s, const KmArgs& a, int single) {
        hipLaunchKernelGGL(km_sse<LP>, g, dim3(KT), 0, s, a, single);
    }
};

struct Dispatch {
    void (*stats)(dim3, hipStream_t, const KmArgs&);
    void (*far)(dim3, hipStream_t, const KmArgs&, int);
    void (*lloyd)(dim3, hipStream_t, const KmArgs&, int, int);
    void (*sse)(dim3, hipStream_t, const KmArgs&, int);
};

template <int LP>
Dispatch make_dispatch() {
    return Dispatch{&Passes<LP>::stats, &Passes<LP>::far, &Passes<LP>::lloyd, &Passes<LP>::sse};
}

Dispatch dispatch_for(int rho) {
    switch (lanes_per_point(rho)) {
        case 1: return make_dispatch<1>();
        case 2: return make_dispatch<2>();
        case 4: return make_dispatch<4>();
        case 8: return make_dispatch<8>();
        case 16: return make_dispatch<16>();
        case 32: return make_dispatch<32>();
        default: return make_dispatch<64>();
    }
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

size_t kmeans_workspace(long long N, int rho, int K) {
    Arena probe;  // counts only
    carve(probe, N, rho, K);
    return probe.used;
}

void kmeans_run(Ctx& c, Arena& ws, const float* guide, int rho, long long N, int K, int max_iter,
                int* labels, KmResult& out) {
    FHD_REQUIRE(N >= 1 && N < (1LL << 31), FHD_EINVAL, "image too large for clustering");
    FHD_REQUIRE(rho >= 1 && rho <= FHD_MAX_RHO, FHD_EUNSUPPORTED, "guide dimension out of range");
    FHD_REQUIRE(K >= 1 && K <= FHD_MAX_K, FHD_EINVAL, "K out of range");
    FHD_REQUIRE(max_iter >= 1, FHD_EINVAL, "kmeans_max_iter must be >= 1");
    KmBuffers B = carve(ws, N, rho, K);
    const Dispatch D = dispatch_for(rho);
    const long long CH = chunk_points(rho);
    hipStream_t st = c.stream;

    // pinned staging: block table + per-job state
    const size_t stage_bytes = align_up(sizeof(int4) * B.maxBlocks, 256) +
                               align_up(sizeof(int) * B.maxJobs * JI_W, 256) +
                               3 * align_up(sizeof(double) * B.maxJobs * rho, 256) +
                               align_up(sizeof(double) * B.maxJobs * JD_W, 256);
    char* hs = static_cast<char*>(c.host_stage(0, stage_bytes));
    Stage H;
    {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            char* p = hs + off;
            off += align_up(bytes, 256);
            return p;
        };
        H.btab = reinterpret_cast<int4*>(take(sizeof(int4) * B.maxBlocks));
        H.ji = reinterpret_cast<int*>(take(sizeof(int) * B.maxJobs * JI_W));
        H.jm = reinterpret_cast<double*>(take(sizeof(double) * B.maxJobs * rho));
        H.ca = reinterpret_cast<double*>(take(sizeof(double) * B.maxJobs * rho));
        H.cb = reinterpret_cast<double*>(take(sizeof(double) * B.maxJobs * rho));
        H.jd = reinterpret_cast<double*>(take(sizeof(double) * B.maxJobs * JD_W));
    }

    KmArgs a{};
    for (int q = 0; q < 2; ++q) {
        a.pts[q] = B.pts[q];
        a.idx[q] = B.idx[q];
        a.side[q] = B.side[q];
    }
    a.btab = B.btab;
    a.blkA = B.blkA;
    a.part = B.part;
    a.ji = B.ji;
    a.jm = B.jm;
    a.ca = B.ca;
    a.cb = B.cb;
    a.jd = B.jd;
    a.done = B.done;
    a.rho = rho;
    a.pw = 4 * rho + 8;

    hipEvent_t t_begin = c.stage_begin();
    FHD_HIP(hipMemsetAsync(B.done, 0, sizeof(unsigned) * B.maxJobs, st));
    hipLaunchKernelGGL(km_pack, dim3((unsigned)((N + KT - 1) / KT)), dim3(KT), 0, st, guide, rho,
                       N, B.pts[0], B.idx[0]);
    FHD_HIP(hipGetLastError());

    // Upload jobs (ranges of leaves) and their block table; returns #blocks.
    auto upload = [&](const std::vector<Leaf*>& jobs, bool with_mean, bool label_rank) -> int {
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
                H.btab[nb++] = make_int4((int)j, s0, cnt, label_rank ? (int)j : q);
            }
            if (with_mean)
                for (int t = 0; t < rho; ++t) H.jm[j * rho + t] = L.mean[t];
        }
        FHD_REQUIRE(nb <= B.maxBlocks, FHD_EINVAL, "internal: block table overflow");
        FHD_HIP(hipMemcpyAsync(B.btab, H.btab, sizeof(int4) * nb, hipMemcpyHostToDevice, st));
        FHD_HIP(hipMemcpyAsync(B.ji, H.ji, sizeof(int) * JI_W * jobs.size(), hipMemcpyHostToDevice,
                               st));
        if (with_mean)
            FHD_HIP(hipMemcpyAsync(B.jm, H.jm, sizeof(double) * rho * jobs.size(),
                                   hipMemcpyHostToDevice, st));
        return nb;
    };

    // ---- root: centroid, SSE, splittable
    std::vector<Leaf> store;
    store.reserve(4 * (size_t)K + 4);
    store.emplace_back();
    Leaf* root = &store.back();
    root->heap = "1";
    root->start = 0;
    root->count = (int)N;
    root->buf = 0;
    {
        std::vector<Leaf*> jobs{root};
        const int nb = upload(jobs, false, false);
        D.stats(dim3(nb), st, a);
        D.sse(dim3(nb), st, a, 1);
        FHD_HIP(hipGetLastError());
        FHD_HIP(hipMemcpyAsync(H.jm, B.jm, sizeof(double) * rho, hipMemcpyDeviceToHost, st));
        FHD_HIP(hipMemcpyAsync(H.jd, B.jd, sizeof(double) * JD_W, hipMemcpyDeviceToHost, st));
        FHD_HIP(hipStreamSynchronize(st));
        root->mean.assign(H.jm, H.jm + rho);
        root->splittable = H.jd[JD_SPLA] != 0.0;
        root->sse = root->splittable ? H.jd[JD_SSEA] : 0.0;
    }

    std::vector<Leaf*> leaves{root};
    int rounds = 0, splits = 0;
    auto rank_less = [](const Leaf* x, const Leaf* y) {
        if (x->sse != y->sse) return x->sse > y->sse;
        return heap_less(x->heap, y->heap);
    };
    while ((int)leaves.size() < K) {
        // leaves the greedy rule can still pick: the top (K - #leaves) splittable ones
        std::vector<Leaf*> cand;
        for (Leaf* L : leaves)
            if (L->splittable && L->sse > 0.0) cand.push_back(L);
        if (cand.empty()) break;
        std::sort(cand.begin(), cand.end(), rank_less);
        const size_t budget = (size_t)K - leaves.size();
        if (cand.size() > budget) cand.resize(budget);
        std::vector<Leaf*> jobs;
        for (Leaf* L : cand)
            if (!L->has_split) jobs.push_back(L);
        if (!jobs.empty()) {
            FHD_REQUIRE((int)jobs.size() <= B.maxJobs, FHD_EINVAL, "internal: too many jobs");
            const int nb = upload(jobs, true, false);
            const dim3 g(nb);
            D.far(g, st, a, 0);
            D.far(g, st, a, 1);
            for (int it = 0; it < max_iter; ++it) D.lloyd(g, st, a, it, max_iter);
            D.sse(g, st, a, 0);
            hipLaunchKernelGGL(km_scatter, g, dim3(KT), 0, st, a);
            FHD_HIP(hipGetLastError());
            const size_t J = jobs.size();
            FHD_HIP(hipMemcpyAsync(H.ca, B.ca, sizeof(double) * rho * J, hipMemcpyDeviceToHost, st));
            FHD_HIP(hipMemcpyAsync(H.cb, B.cb, sizeof(double) * rho * J, hipMemcpyDeviceToHost, st));
            FHD_HIP(hipMemcpyAsync(H.jd, B.jd, sizeof(double) * JD_W * J, hipMemcpyDeviceToHost, st));
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
                FHD_REQUIRE(L.nA > 0 && L.nB > 0 && L.nA + L.nB == L.count, FHD_ENUMERIC,
                            "internal: degenerate 2-means split");
            }
            ++rounds;
            splits += (int)J;
        }
        // commit greedily while the best leaf's split is known
        while ((int)leaves.size() < K) {
            Leaf* best = nullptr;
            for (Leaf* L : leaves)
                if (L->splittable && L->sse > 0.0 && (best == nullptr || rank_less(L, best))) best = L;
            if (best == nullptr || !best->has_split) break;
            store.emplace_back();
            Leaf* A = &store.back();
            store.emplace_back();
            Leaf* Bc = &store.back();
            A->heap = best->heap + "0";
            A->start = best->start;
            A->count = best->nA;
            A->buf = 1 - best->buf;
            A->mean = best->meanA;
            A->sse = best->sseA;
            A->splittable = best->splA;
            Bc->heap = best->heap + "1";
            Bc->start = best->start + best->nA;
            Bc->count = best->nB;
            Bc->buf = 1 - best->buf;
            Bc->mean = best->meanB;
            Bc->sse = best->sseB;
            Bc->splittable = best->splB;
            leaves.erase(std::find(leaves.begin(), leaves.end(), best));
            leaves.push_back(A);
            leaves.push_back(Bc);
        }
        bool any = false;
        for (Leaf* L : leaves) any = any || (L->splittable && L->sse > 0.0);
        if (!any) break;
    }

    std::sort(leaves.begin(), leaves.end(),
              [](const Leaf* x, const Leaf* y) { return heap_less(x->heap, y->heap); });
    out.K_eff = (int)leaves.size();
    out.rounds = rounds;
    out.splits = splits;
    out.E_K = 0.0;
    out.centers.assign((size_t)out.K_eff * rho, 0.0);
    for (int k = 0; k < out.K_eff; ++k) {
        out.E_K += leaves[k]->sse;
        for (int t = 0; t < rho; ++t) out.centers[(size_t)k * rho + t] = leaves[k]->mean[t];
    }
    if (labels != nullptr) {
        std::vector<Leaf*> jobs(leaves.begin(), leaves.end());
        const int nb = upload(jobs, false, true);
        hipLaunchKernelGGL(km_labels, dim3(nb), dim3(KT), 0, st, a, labels);
        FHD_HIP(hipGetLastError());
    }
    c.stage_end(FHD_STAGE_CLUSTER, t_begin);
    c.stage_done(0);
}

}  // namespace fhd
