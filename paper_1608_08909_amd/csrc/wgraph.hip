// Graphs with edge lengths: Algorithm 1's general input (every edge has a
// positive length; unit lengths give back the unweighted model).
//
// - Distances are shortest-path lengths, the sum along a path taken from the
//   source outwards in FP64: the least solution of d(s) = 0,
//   d(v) = min over neighbours u of (d(u) + len(u, v)).  A label-correcting
//   search reaches exactly that solution whatever the order of its
//   relaxations (every sum is monotone in d(u)), so the result is bit for bit
//   Dijkstra's.
// - Edge terms carry w_ij = len^-2; pivot terms exist for every pivot that is
//   neither i nor a neighbour of i, with w'_ip = s / d_ip^2,
//   s = |{ j in R(p) : delta_j <= d_ip / 2 }| (Section 3 with real distances),
//   one weight per (pivot, node) since s no longer depends on d alone through
//   an integer table.
// - Regions follow rule R1 with levels at the distinct values of delta.
#include <float.h>

#include <hipcub/hipcub.hpp>

#include <vector>

#include "ssm_internal.h"
#include "wave.h"

struct ssm_wterms {
    int device = 0;
    int32_t n = 0, k = 0, nnz = 0;
    void* arena = nullptr;      // one allocation holding every buffer below
    int32_t* pivots = nullptr;  // [k]
    double* dist = nullptr;     // [k][n]
    double* delta = nullptr;    // [n]
    int32_t* region = nullptr;  // [n]
    double* w64 = nullptr;      // [k][n] adapted weights, 0 where no term
    float2* wd32 = nullptr;     // [k][n] (w', w' d) in FP32
    double* den64 = nullptr;    // [n]
    float* den32 = nullptr;     // [n]
    float2* wl32 = nullptr;     // [nnz] (len^-2, len^-1) in FP32
    void* xtmp = nullptr;       // [n][2] doubles: second Jacobi buffer
};

namespace ssm {

constexpr int kSsspBlock = 1024;
constexpr int kSsspLanes = 8;  // lanes per frontier node in the search
constexpr size_t kSsspLdsBits = 128 * 1024;  // largest LDS of the three near-far bitmaps (n <= 349504)

// Variant sssp_nearfar = -1: the plain label-correcting order.
static bool nearfar_off() { return variant("sssp_nearfar") == -1; }
constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;  // +inf; non-negative doubles order as their bits

__device__ __forceinline__ double ld_dist(const unsigned long long* D, int v) {
    return __longlong_as_double((long long)__hip_atomic_load(D + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Label-correcting search from src over D (bits of non-negative doubles):
// each round relaxes the arcs of the nodes whose distance dropped in the
// previous round; a node joins the next round once (stamp = round number,
// rounds numbered from *round upward across calls, so stamp never needs a
// reset).  The values already in D stay as upper bounds: with +inf
// everywhere the search is a plain one; max/min passes its m, which the
// search lowers to min(m, d_src) (a node whose bound is not beaten is not
// expanded: nothing beyond it can improve).  One workgroup; qa and qb hold n
// ints each.
__device__ void sssp_body(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ len, int src, unsigned long long* D, int* stamp, int* qa,
                          int* qb, int* round) {
    __shared__ int s_next;
    __shared__ int s_round;
    if (threadIdx.x == 0) {
        atomicMin(D + src, 0ull);
        s_round = *round;
        qa[0] = src;
        s_next = 0;
    }
    __syncthreads();
    int r = s_round, cnt = 1;
    int* cur = qa;
    int* nxt = qb;
    // kSsspLanes lanes per frontier node, each over every kSsspLanes-th arc
    const int sub = threadIdx.x % kSsspLanes, grp = threadIdx.x / kSsspLanes, ngrp = blockDim.x / kSsspLanes;
    while (cnt > 0) {
        ++r;
        for (int q = grp; q < cnt; q += ngrp) {
            const int u = cur[q];
            const double du = ld_dist(D, u);
            for (int e = rp[u] + sub; e < rp[u + 1]; e += kSsspLanes) {
                const int v = ci[e];
                const unsigned long long nb = (unsigned long long)__double_as_longlong(du + len[e]);
                const unsigned long long old = atomicMin(D + v, nb);
                if (nb < old && atomicExch(stamp + v, r) != r) nxt[atomicAdd(&s_next, 1)] = v;
            }
        }
        __syncthreads();  // every append of the round is done
        cnt = s_next;
        __syncthreads();  // every thread has read the count
        if (threadIdx.x == 0) s_next = 0;
        __syncthreads();  // the reset precedes the next round's appends
        int* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (threadIdx.x == 0) *round = r + 1;
    __syncthreads();
}

// The same least fixed point in near-far order: a relaxed node whose new
// value is below the threshold joins the next round (near), any other joins
// the far list (once: a far bit per node).  When a round leaves nothing near,
// the threshold rises by delta (at least the largest edge length, so the
// next band is never empty) and one pass over the far list drops the nodes
// already expanded (value below the old threshold), moves those now below
// the threshold to the frontier and keeps the rest.  Each node is expanded
// about once instead of once per improvement.  qa, qb, fa, fb hold n ints
// each; sb: three bitmaps of ceil(n / 32) words in LDS (near, alternating
// by round, then far).
__device__ void sssp_nearfar(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ len, int src, unsigned long long* D, int* qa, int* qb,
                             int* fa, int* fb, unsigned* sb, double delta) {
    // near rounds count their appends into s_cnt[r % 3]: round r clears the
    // slot of round r + 1 (last read after round r - 2's barrier) and the
    // bitmap of round r + 1 (last used in round r - 1), so one barrier per
    // round suffices
    __shared__ int s_cnt[3], s_far, s_mv, s_keep;
    const int nbw = (n + 31) / 32;
    unsigned* farb = sb + 2 * nbw;
    for (int w = threadIdx.x; w < 3 * nbw; w += blockDim.x) sb[w] = 0u;
    if (threadIdx.x == 0) {
        atomicMin(D + src, 0ull);
        qa[0] = src;
        s_cnt[0] = s_cnt[1] = s_cnt[2] = 0;
        s_far = 0;
        s_mv = 0;
        s_keep = 0;
    }
    __syncthreads();
    int r = 0, cnt = 1;
    int* cur = qa;
    int* nxt = qb;
    int* fcur = fa;
    int* fnxt = fb;
    double thr = delta;
    const int sub = threadIdx.x % kSsspLanes, grp = threadIdx.x / kSsspLanes, ngrp = blockDim.x / kSsspLanes;
    // a node's values never exceed its first, which follows a tree path of
    // fewer than n edges, so after n passes (each raises the threshold by the
    // largest length) nothing stays far; the bound 2 n + 2 only guards the
    // loop
    for (long long pass = 0; pass <= 2LL * n + 2; ++pass) {
        while (cnt > 0) {
            ++r;
            int* cntr = &s_cnt[r % 3];
            if (threadIdx.x == 0) s_cnt[(r + 1) % 3] = 0;
            unsigned* other = sb + ((r + 1) & 1) * nbw;
            for (int w = threadIdx.x; w < nbw; w += blockDim.x) other[w] = 0u;
            unsigned* bits = sb + (r & 1) * nbw;
            for (int q = grp; q < cnt; q += ngrp) {
                const int u = cur[q];
                const double du = ld_dist(D, u);
                for (int e = rp[u] + sub; e < rp[u + 1]; e += kSsspLanes) {
                    const int v = ci[e];
                    const double dv = du + len[e];
                    const unsigned long long nb = (unsigned long long)__double_as_longlong(dv);
                    const unsigned long long old = atomicMin(D + v, nb);
                    if (nb < old) {
                        const unsigned bit = 1u << (v & 31);
                        if (dv < thr) {
                            if (!(atomicOr(bits + (v >> 5), bit) & bit)) nxt[atomicAdd(cntr, 1)] = v;
                        } else if (!(atomicOr(farb + (v >> 5), bit) & bit)) {
                            fcur[atomicAdd(&s_far, 1)] = v;
                        }
                    }
                }
            }
            __syncthreads();  // every append (and clear) of the round is done
            cnt = *cntr;
            int* t = cur;
            cur = nxt;
            nxt = t;
        }
        // nothing near: next band, one pass over the far list
        const int nfar = s_far;
        if (nfar == 0) break;  // uniform (read after the last barrier)
        const double lo = thr;
        thr += delta;
        for (int q = threadIdx.x; q < nfar; q += blockDim.x) {
            const int v = fcur[q];
            const double dv = ld_dist(D, v);
            const unsigned bit = 1u << (v & 31);
            if (dv < thr) {
                atomicAnd(farb + (v >> 5), ~bit);
                if (dv >= lo) cur[atomicAdd(&s_mv, 1)] = v;  // below lo: expanded already
            } else {
                fnxt[atomicAdd(&s_keep, 1)] = v;
            }
        }
        __syncthreads();  // the pass is done
        cnt = s_mv;
        const int kept = s_keep;
        __syncthreads();  // every thread has read the counts
        if (threadIdx.x == 0) {
            s_mv = 0;
            s_far = kept;
            s_keep = 0;
        }
        __syncthreads();  // the resets precede the next round
        int* t = fcur;
        fcur = fnxt;
        fnxt = t;
    }
}

// Block b: the full search from pivots[b] into row b of D (pre-filled with
// +inf); stamp, qa, qb: n ints per block (stamp unused with LBITS).
//   NF: near-far order with its bitmaps in LDS; q holds 4 n ints per block
//   and *delta the band width.  Otherwise the plain search with global
//   stamps; q holds 2 n ints per block.
template <bool NF>
__global__ __launch_bounds__(kSsspBlock) void k_sssp_rows(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci, const double* __restrict__ len,
                                                          const int* __restrict__ pivots, unsigned long long* D,
                                                          int* stamp, int* q, int* rounds,
                                                          const unsigned long long* __restrict__ delta) {
    extern __shared__ unsigned sbits[];
    const int b = blockIdx.x;
    if (NF) {
        int* qb = q + (size_t)b * 4 * n;
        sssp_nearfar(n, rp, ci, len, pivots[b], D + (size_t)b * n, qb, qb + n, qb + 2 * (size_t)n,
                     qb + 3 * (size_t)n, sbits, __longlong_as_double((long long)*delta));
    } else {
        sssp_body(n, rp, ci, len, pivots[b], D + (size_t)b * n, stamp + (size_t)b * n, q + (size_t)b * 2 * n,
                  q + (size_t)b * 2 * n + n, rounds + b);
    }
}

// out[0] = bits of the largest length (pre-filled with 0; positive doubles
// order as their bits); *bad = 1 if a length is not positive and finite.
__global__ void k_len_check(long long count, const double* __restrict__ len, unsigned long long* out, int* bad) {
    unsigned long long b = 0;
    bool ok = true;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < count;
         q += (long long)gridDim.x * blockDim.x) {
        const double v = len[q];
        ok = ok && v > 0.0 && v <= DBL_MAX;  // false for NaN too
        const unsigned long long u = (unsigned long long)__double_as_longlong(v);
        b = v > 0.0 && u > b ? u : b;
    }
    b = wave_max(b);
    if (lane_id() == 0) atomicMax(out, b);
    if (!ok) *bad = 1;
}

// *delta *= c (bits of a positive double).
__global__ void k_band_scale(unsigned long long* delta, double c) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *delta = (unsigned long long)__double_as_longlong(c * __longlong_as_double((long long)*delta));
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, long long count) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < count;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

__global__ void k_fill_i32(int* p, int v, long long count) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < count;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

// max/min sp with lengths, one workgroup: m = min over the chosen pivots'
// distances (each search pruned by m itself), next pivot = largest m, lowest
// id on ties.  status[0] = 1 if the first search leaves a node unreached.
//   NF: near-far searches (fa, fb: n ints each, *delta the band width).
template <bool NF>
__global__ __launch_bounds__(kSsspBlock) void k_select_w(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double* __restrict__ len,
                                                         int k, int first, int* pivots, unsigned long long* m,
                                                         int* stamp, int* qa, int* qb, int* fa, int* fb, int* round,
                                                         int* status, const unsigned long long* __restrict__ delta) {
    extern __shared__ unsigned sbits[];
    __shared__ double s_bv[kSsspBlock / kWave];
    __shared__ int s_bi[kSsspBlock / kWave];
    __shared__ int s_src;
    if (threadIdx.x == 0) s_src = first;
    __syncthreads();
    for (int t = 0; t < k; ++t) {
        const int src = s_src;
        if (threadIdx.x == 0) pivots[t] = src;
        if (NF)
            sssp_nearfar(n, rp, ci, len, src, m, qa, qb, fa, fb, sbits, __longlong_as_double((long long)*delta));
        else
            sssp_body(n, rp, ci, len, src, m, stamp, qa, qb, round);
        if (t + 1 >= k && t != 0) break;
        // argmax of m: strict comparison over ascending ids per thread keeps
        // the lowest id among equal values (eight loads in flight)
        double bv = -1.0;
        int bi = n;
        constexpr int U = 8;
        for (int i0 = threadIdx.x; i0 < n; i0 += U * blockDim.x) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                v[u] = i < n ? ld_dist(m, i) : -1.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (v[u] > bv) {
                    bv = v[u];
                    bi = i0 + u * (int)blockDim.x;
                }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane_id() == 0) {
            s_bv[threadIdx.x / kWave] = bv;
            s_bi[threadIdx.x / kWave] = bi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < (int)blockDim.x / kWave; ++w)
                if (s_bv[w] > bv || (s_bv[w] == bv && s_bi[w] < bi)) {
                    bv = s_bv[w];
                    bi = s_bi[w];
                }
            if (t == 0 && bv == __longlong_as_double((long long)kInfBits)) status[0] = 1;
            s_src = bi;
        }
        __syncthreads();
        if (t == 0 && status[0]) break;  // uniform after the barrier
    }
}

// Any +inf in the k x n table: flag[0] = 1.
__global__ void k_any_inf(long long total, const unsigned long long* __restrict__ D, int* flag) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x)
        if (D[q] == kInfBits) flag[0] = 1;
}

// ------------------------------------------------------------- regions

// Per node: delta, the number of candidates, the first one; singles join it
// at once (region), tied nodes get -1.  flags[i] = tied.
__global__ void k_wreg_scan(int n, int k, const double* __restrict__ dist, double* __restrict__ delta,
                            int* __restrict__ region, int* __restrict__ tied) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double best = __longlong_as_double((long long)kInfBits);
        int cnt = 0, at = 0;
        constexpr int U = 8;  // loads in flight; ranks compared in ascending order
        for (int t0 = 0; t0 < k; t0 += U) {
            double dv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) dv[j] = t0 + j < k ? dist[(size_t)(t0 + j) * n + i] : 0.0;
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (t0 + j >= k) break;
                const double d = dv[j];
                if (d < best) {
                    best = d;
                    cnt = 1;
                    at = t0 + j;
                } else if (d == best) {
                    ++cnt;
                }
            }
        }
        delta[i] = best;
        region[i] = cnt == 1 ? at : -1;
        tied[i] = cnt > 1;
    }
}

// Sort keys: delta bits and region per node; single nodes only when
// `singles` (others get the key past every region, k).
__global__ void k_wreg_keys(int n, int k, const double* __restrict__ delta, const int* __restrict__ region,
                            bool singles, unsigned long long* __restrict__ dkey, int* __restrict__ rval) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        dkey[i] = (unsigned long long)__double_as_longlong(delta[i]);
        const int r = region[i];
        rval[i] = singles && r < 0 ? k : r;
    }
}

// Region segments of a (region, delta)-sorted array: start[t] = first index
// of region t (start[k] = end of the regions' part).
__global__ void k_wreg_starts(int n, int k, const int* __restrict__ rsorted, int* __restrict__ start) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q <= n; q += gridDim.x * blockDim.x) {
        const int a = q > 0 ? rsorted[q - 1] : -1, b = q < n ? rsorted[q] : k + 1;
        for (int t = a + 1; t <= min(b, k); ++t) start[t] = q;
    }
}

// Number of entries <= x in the ascending segment [lo, hi) of keys (bits of
// non-negative doubles).
__device__ __forceinline__ int count_le(const unsigned long long* __restrict__ keys, int lo, int hi, double x) {
    const unsigned long long xb = (unsigned long long)__double_as_longlong(x);
    int a = lo, b = hi;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (keys[mid] <= xb)
            a = mid + 1;
        else
            b = mid;
    }
    return a - lo;
}

// Tied nodes in (delta, id) order, one workgroup: a level (equal delta)
// decides against size snapshots = single members at delta <= level (from
// the singles' sorted segments) + tied members of earlier levels; the lowest
// (snapshot, rank) wins.
__global__ __launch_bounds__(1024) void k_wreg_ties(int n, int k, int ntied, const int* __restrict__ tied_ids,
                                                    const unsigned long long* __restrict__ tied_keys,
                                                    const double* __restrict__ dist,
                                                    const unsigned long long* __restrict__ skeys,
                                                    const int* __restrict__ sstart, int* __restrict__ region) {
    extern __shared__ int tcount[];  // [k]
    __shared__ int s_end;
    for (int t = threadIdx.x; t < k; t += blockDim.x) tcount[t] = 0;
    __syncthreads();
    for (int a = 0; a < ntied;) {
        // the level: [a, end) with equal keys
        if (threadIdx.x == 0) {
            int e = a + 1;
            while (e < ntied && tied_keys[e] == tied_keys[a]) ++e;
            s_end = e;
        }
        __syncthreads();
        const int end = s_end;
        const double L = __longlong_as_double((long long)tied_keys[a]);
        for (int q = a + (int)threadIdx.x; q < end; q += blockDim.x) {
            const int i = tied_ids[q];
            int pick = -1;
            long long best = 0;
            for (int t = 0; t < k; ++t) {
                if (dist[(size_t)t * n + i] != L) continue;
                const long long snap = (long long)count_le(skeys, sstart[t], sstart[t + 1], L) + tcount[t];
                if (pick < 0 || snap < best) {
                    pick = t;
                    best = snap;
                }
            }
            region[i] = pick;
        }
        __syncthreads();
        for (int q = a + (int)threadIdx.x; q < end; q += blockDim.x) atomicAdd(&tcount[region[tied_ids[q]]], 1);
        __syncthreads();
        a = end;
    }
}

// ------------------------------------------------------------- terms

// w[t][i] = s / d^2 for pivot p_t not i and not a neighbour of i, with s the
// members of region t at delta <= d / 2 (count in the region's sorted
// segment); FP32 pair (w', w' d).
__global__ void k_wterms(int n, int k, const int* __restrict__ rp, const int* __restrict__ ci,
                         const int* __restrict__ pivots, const double* __restrict__ dist,
                         const unsigned long long* __restrict__ akeys, const int* __restrict__ astart,
                         double* __restrict__ w64, float2* __restrict__ wd32) {
#pragma clang fp contract(off)
    const long long total = (long long)k * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(q / n), i = (int)(q % n);
        const int p = pivots[t];
        bool term = i != p;
        for (int e = rp[i]; e < rp[i + 1] && term; ++e) term = ci[e] != p;
        const double d = dist[q];
        double val = 0.0;
        if (term) {
            const int s = count_le(akeys, astart[t], astart[t + 1], d / 2.0);
            val = (double)s / (d * d);
        }
        w64[q] = val;
        wd32[q] = make_float2((float)val, (float)(val * d));
    }
}

// den_i = sum over i's arcs in CSR order of len^-2, then over ranks
// ascending of w[t][i]; FP32 copies; the arcs' FP32 pairs (len^-2, len^-1).
__global__ void k_wden(int n, int k, const int* __restrict__ rp, const double* __restrict__ len,
                       const double* __restrict__ w64, double* __restrict__ den64, float* __restrict__ den32,
                       float2* __restrict__ wl32) {
#pragma clang fp contract(off)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const double we = 1.0 / (len[e] * len[e]);
            s += we;
            wl32[e] = make_float2((float)we, (float)(we * len[e]));
        }
        constexpr int U = 8;  // loads in flight; the sum keeps ascending ranks
        for (int t0 = 0; t0 < k; t0 += U) {
            double wv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) wv[j] = t0 + j < k ? w64[(size_t)(t0 + j) * n + i] : 0.0;
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (t0 + j < k) s += wv[j];
        }
        den64[i] = s;
        den32[i] = (float)s;
    }
}

// ------------------------------------------------------------- sweeps

// FP64 sweep in the oracle's order: positive-distance neighbour votes
// len^-2 (x_j + len (x_i - x_j) / r) in CSR order, then the zero-distance
// ones len^-2 x_i, then pivot terms by ascending rank, w (x_p + d (x_i - x_p)
// / r) or w x_p at r = 0.
__global__ __launch_bounds__(256) void k_wsweep_f64(int n, int k, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const double* __restrict__ len,
                                                    const double2* __restrict__ xo, double2* __restrict__ xn,
                                                    const int* __restrict__ piv, const double* __restrict__ dist,
                                                    const double* __restrict__ w64,
                                                    const double* __restrict__ den) {
#pragma clang fp contract(off)
    extern __shared__ double2 sP[];
    for (int t = threadIdx.x; t < k; t += blockDim.x) sP[t] = xo[piv[t]];
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double2 xv = xo[i];
        const double xi = xv.x, yi = xv.y;
        double nx = 0.0, ny = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const double2 xj = xo[ci[e]];
            const double dx = xi - xj.x, dy = yi - xj.y;
            const double r = sqrt(dx * dx + dy * dy);
            if (r > 0.0) {
                const double we = 1.0 / (len[e] * len[e]);
                nx += we * (xj.x + (len[e] * dx) / r);
                ny += we * (xj.y + (len[e] * dy) / r);
            }
        }
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const double2 xj = xo[ci[e]];
            const double dx = xi - xj.x, dy = yi - xj.y;
            const double r = sqrt(dx * dx + dy * dy);
            if (!(r > 0.0)) {
                const double we = 1.0 / (len[e] * len[e]);
                nx += we * xi;
                ny += we * yi;
            }
        }
        for (int t = 0; t < k; ++t) {
            const double wt = w64[(size_t)t * n + i];
            if (wt == 0.0) continue;
            const double d = dist[(size_t)t * n + i];
            const double2 p = sP[t];
            const double dx = xi - p.x, dy = yi - p.y;
            const double r = sqrt(dx * dx + dy * dy);
            double vx = p.x, vy = p.y;
            if (r > 0.0) {
                vx = p.x + d * dx / r;
                vy = p.y + d * dy / r;
            }
            nx += wt * vx;
            ny += wt * vy;
        }
        const double dn = den[i];
        xn[i] = make_double2(nx / dn, ny / dn);
    }
}

// FP32 sweep, displacement form: x_i' = x_i + (sum_q f_q (x_q - x_i)) / den_i
// with f = w - (w d) / r per term (a term with w = 0 adds exactly 0).  A
// block is kWSplit waves on the same 64 nodes: wave w sums the pivot terms
// of ranks t = w (mod kWSplit), the last wave also the neighbour terms in
// CSR order; wave 0 adds the partials in a fixed order.  The (w', w' d) pairs
// are read coalesced, rank-major, four ranks ahead.
constexpr int kWSplit = 4;

__global__ __launch_bounds__(64 * kWSplit) void k_wsweep_f32(int n, int k, const int* __restrict__ rp,
                                                             const int* __restrict__ ci, const float2* __restrict__ wl,
                                                             const float2* __restrict__ xo, float2* __restrict__ xn,
                                                             const int* __restrict__ piv,
                                                             const float2* __restrict__ wd,
                                                             const float* __restrict__ den) {
    extern __shared__ float2 sQ[];  // [k] pivot coordinates, then [kWSplit][64] partials
    float2* part = sQ + k;
    for (int t = threadIdx.x; t < k; t += blockDim.x) sQ[t] = xo[piv[t]];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const float tiny = 1e-30f;
    const int nchunks = (n + 63) / 64;
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {  // uniform over the block
        __syncthreads();  // pivots staged; the previous chunk's partials consumed
        const int i = c * 64 + lane;
        float ax = 0.f, ay = 0.f;
        float2 xi = make_float2(0.f, 0.f);
        if (i < n) {
            xi = xo[i];
            if (w == kWSplit - 1) {
                for (int e = rp[i]; e < rp[i + 1]; ++e) {
                    const float2 xj = xo[ci[e]];
                    const float2 f01 = wl[e];
                    const float dx = xj.x - xi.x, dy = xj.y - xi.y;
                    const float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
                    const float f = fmaf(-f01.y, inv, f01.x);
                    ax += f * dx;
                    ay += f * dy;
                }
            }
            const float2* __restrict__ wp = wd + i;
            float2 buf[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = w + u * kWSplit;
                buf[u] = t < k ? wp[(size_t)t * n] : make_float2(0.f, 0.f);
            }
            for (int t0 = w; t0 < k; t0 += 4 * kWSplit) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = t0 + u * kWSplit;
                    if (t >= k) break;
                    const float2 f01 = buf[u];
                    const int tn = t + 4 * kWSplit;
                    if (tn < k) buf[u] = wp[(size_t)tn * n];
                    const float2 pv = sQ[t];
                    const float dx = pv.x - xi.x, dy = pv.y - xi.y;
                    const float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
                    const float f = fmaf(-f01.y, inv, f01.x);
                    ax += f * dx;
                    ay += f * dy;
                }
            }
        }
        part[w * 64 + lane] = make_float2(ax, ay);
        __syncthreads();
        if (w == 0 && i < n) {
            float sx = 0.f, sy = 0.f;
#pragma unroll
            for (int q = 0; q < kWSplit; ++q) {
                const float2 o = part[q * 64 + lane];
                sx += o.x;
                sy += o.y;
            }
            const float dn = den[i];
            xn[i] = make_float2(xi.x + sx / dn, xi.y + sy / dn);
        }
    }
}

__global__ void k_wround(int n, const double2* __restrict__ a, float2* __restrict__ b) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// Per-block partials of s'(x) with lengths (FP64): edges j > i, then every
// pivot term of i.
template <typename T2>
__global__ __launch_bounds__(256) void k_wstress(int n, int k, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const double* __restrict__ len, const T2* __restrict__ x,
                                                 const int* __restrict__ piv, const double* __restrict__ dist,
                                                 const double* __restrict__ w64, double* __restrict__ partials) {
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double xi = (double)x[i].x, yi = (double)x[i].y;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = ci[e];
            if (j <= i) continue;
            const double dx = xi - (double)x[j].x, dy = yi - (double)x[j].y;
            const double r = sqrt(dx * dx + dy * dy);
            acc += (r - len[e]) * (r - len[e]) / (len[e] * len[e]);
        }
        for (int t = 0; t < k; ++t) {
            const double wt = w64[(size_t)t * n + i];
            if (wt == 0.0) continue;
            const int p = piv[t];
            const double dx = xi - (double)x[p].x, dy = yi - (double)x[p].y;
            const double r = sqrt(dx * dx + dy * dy);
            const double d = dist[(size_t)t * n + i];
            acc += wt * (r - d) * (r - d);
        }
    }
    __shared__ double red[256 / kWave];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// keys[q] = delta bits of node ids[q].
__global__ void k_gather_dkeys(int count, const int* __restrict__ ids, const double* __restrict__ delta,
                               unsigned long long* __restrict__ keys) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < count; q += gridDim.x * blockDim.x)
        keys[q] = (unsigned long long)__double_as_longlong(delta[ids[q]]);
}

// ------------------------------------------------------------- host

namespace {

// Radix sort of (key, value) pairs on bits [0, bits) into the out arrays.
template <typename K, typename V>
hipError_t sort_pairs(const K* kin, K* kout, const V* vin, V* vout, int count, int bits, hipStream_t s) {
    size_t tb = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, kin, kout, vin, vout, count, 0, bits, s);
    if (e != hipSuccess) return e;
    void* tmp = nullptr;
    if (salloc(&tmp, std::max<size_t>(tb, 1)) != SSM_OK) return hipErrorOutOfMemory;
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, vin, vout, count, 0, bits, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    sfree(tmp);
    return e != hipSuccess ? e : e2;
}

// Device check of the lengths: *delta = c times the largest one (the band
// width of the near-far searches; an integer c >= 1 keeps their far-pass
// bound); SSM_E_INVAL if a length is not positive and finite.  Synchronizes.
ssm_status length_band(const ssm_csr* g, const double* len, unsigned long long* delta, int* bad, int c,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, delta, 0ull, 1LL);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, bad, 0, 1LL);
    // few blocks: each ends in an atomic on the same word
    hipLaunchKernelGGL(k_len_check, dim3(std::max(1, std::min(div_up(g->nnz, 1024), 128))), dim3(256), 0, s,
                       (long long)g->nnz, len, delta, bad);
    if (const int v = variant("sssp_band")) c = v;  // variant override
    if (c > 1) hipLaunchKernelGGL(k_band_scale, dim3(1), dim3(64), 0, s, delta, (double)c);
    int hb = 0;
    SSM_HIP(hipGetLastError());
    SSM_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    SSM_HIP(hipStreamSynchronize(s));
    if (hb) return fail(SSM_E_INVAL, "edge lengths must be positive and finite");
    return SSM_OK;
}

int bits_for(int v) {  // bits that hold 0 .. v
    int b = 1;
    while ((1LL << b) <= v) ++b;
    return b;
}

}  // namespace

ssm_status select_pivots_w(const ssm_csr* g, const double* len, int32_t k, int32_t first, int32_t* pivots,
                           hipStream_t s) {
    const int n = g->n;
    char* ws = nullptr;
    const size_t bytes = sizeof(unsigned long long) * ((size_t)n + 1) + sizeof(int) * (5 * (size_t)n + 3);
    ssm_status st = salloc((void**)&ws, bytes);
    if (st != SSM_OK) return st;
    unsigned long long* m = (unsigned long long*)ws;
    unsigned long long* delta = m + n;
    int* stamp = (int*)(delta + 1);
    int* qa = stamp + n;
    int* qb = qa + n;
    int* fa = qb + n;
    int* fb = fa + n;
    int* ctl = fb + n;  // round, status, length check
    // many short pruned searches: bands of two lengths (fewer rounds) measured
    // faster than one on MI355X; the full rows take one
    st = length_band(g, len, delta, ctl + 2, 2, s);
    if (st != SSM_OK) {
        (void)hipStreamSynchronize(s);  // idle before the scratch is reused
        sfree(ws);
        return st;
    }
    const int gb = std::min(div_up(n, 256), 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3(gb), dim3(256), 0, s, m, kInfBits, (long long)n);
    hipLaunchKernelGGL(k_fill_i32, dim3(gb), dim3(256), 0, s, stamp, 0, (long long)n);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, ctl, 0, 2LL);
    const size_t lbits = 3 * sizeof(unsigned) * (size_t)((n + 31) / 32);
    if (lbits <= kSsspLdsBits && !nearfar_off()) {
        (void)hipFuncSetAttribute((const void*)k_select_w<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kSsspLdsBits);
        hipLaunchKernelGGL(k_select_w<true>, dim3(1), dim3(kSsspBlock), lbits, s, n, g->row_ptr, g->col_idx, len, k,
                           first, pivots, m, stamp, qa, qb, fa, fb, ctl, ctl + 1, delta);
    } else {
        hipLaunchKernelGGL(k_select_w<false>, dim3(1), dim3(kSsspBlock), 0, s, n, g->row_ptr, g->col_idx, len, k,
                           first, pivots, m, stamp, qa, qb, fa, fb, ctl, ctl + 1, delta);
    }
    hipError_t e = hipGetLastError();
    int hs = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hs, ctl + 1, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "pivot selection (edge lengths)");
    if (hs) return fail(SSM_E_DISCONNECTED, "graph is not connected (the first search missed nodes)");
    return SSM_OK;
}

ssm_status sssp_rows(const ssm_csr* g, const double* len, int32_t k, const int32_t* pivots, double* dist,
                     hipStream_t s) {
    const int n = g->n;
    // rows per launch; each block holds n ints of stamps and 2 n of queues
    // (plain search) or 4 n of queues (near-far)
    const int blocks = std::min(k, 4 * num_cus());
    const size_t lbits = 3 * sizeof(unsigned) * (size_t)((n + 31) / 32);
    const bool nf = lbits <= kSsspLdsBits && !nearfar_off();
    char* ws = nullptr;
    const size_t per_block = nf ? 4 * (size_t)n : 3 * (size_t)n;
    const size_t bytes = sizeof(unsigned long long) + sizeof(int) * (per_block * blocks + blocks + 2);
    ssm_status st = salloc((void**)&ws, bytes);
    if (st != SSM_OK) return st;
    unsigned long long* delta = (unsigned long long*)ws;
    int* q = (int*)(delta + 1);
    int* stamp = nf ? nullptr : q + 2 * (size_t)n * blocks;
    int* rounds = q + per_block * blocks;
    int* flag = rounds + blocks;
    st = length_band(g, len, delta, flag + 1, 1, s);
    if (st != SSM_OK) {
        (void)hipStreamSynchronize(s);  // idle before the scratch is reused
        sfree(ws);
        return st;
    }
    const long long total = (long long)k * n;
    hipLaunchKernelGGL(k_fill_u64, dim3(std::min(div_up(total, 256), 8192)), dim3(256), 0, s,
                       (unsigned long long*)dist, kInfBits, total);
    hipError_t e = hipGetLastError();
    if (nf)
        (void)hipFuncSetAttribute((const void*)k_sssp_rows<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kSsspLdsBits);
    for (int b0 = 0; b0 < k && e == hipSuccess; b0 += blocks) {
        const int nb = std::min(blocks, k - b0);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, rounds, 0, (long long)blocks + 1);
        if (nf) {
            hipLaunchKernelGGL(k_sssp_rows<true>, dim3(nb), dim3(kSsspBlock), lbits, s, n, g->row_ptr, g->col_idx,
                               len, pivots + b0, (unsigned long long*)(dist + (size_t)b0 * n), stamp, q, rounds, delta);
        } else {
            hipLaunchKernelGGL(k_fill_i32, dim3(std::min(div_up((long long)n * nb, 256), 8192)), dim3(256), 0, s,
                               stamp, 0, (long long)n * nb);
            hipLaunchKernelGGL(k_sssp_rows<false>, dim3(nb), dim3(kSsspBlock), 0, s, n, g->row_ptr, g->col_idx, len,
                               pivots + b0, (unsigned long long*)(dist + (size_t)b0 * n), stamp, q, rounds, delta);
        }
        e = hipGetLastError();
    }
    int hf = 0;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_any_inf, dim3(std::min(div_up(total, 256), 4096)), dim3(256), 0, s, total,
                           (const unsigned long long*)dist, flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "shortest paths (edge lengths)");
    if (hf) return fail(SSM_E_DISCONNECTED, "graph is not connected (a search missed nodes)");
    return SSM_OK;
}

// Regions, terms and denominators into t (pivots and dist already there).
static ssm_status build_wterms(const ssm_csr* g, const double* len, ssm_wterms* t, hipStream_t s) {
    const int n = t->n, k = t->k;
    const int gn = std::min(div_up(n, 256), 8192);
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += (b + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_tied = take(sizeof(int) * n), o_ids = take(sizeof(int) * n), o_tids = take(sizeof(int) * n),
                 o_nt = take(sizeof(int) * 2), o_k1 = take(sizeof(unsigned long long) * n),
                 o_k2 = take(sizeof(unsigned long long) * n), o_r1 = take(sizeof(int) * n),
                 o_r2 = take(sizeof(int) * n), o_sk = take(sizeof(unsigned long long) * n),
                 o_ss = take(sizeof(int) * ((size_t)k + 2)), o_tk = take(sizeof(unsigned long long) * n),
                 o_ak = take(sizeof(unsigned long long) * n), o_as = take(sizeof(int) * ((size_t)k + 2));
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, off);
    if (st != SSM_OK) return st;
    int* tied = (int*)(ws + o_tied);
    int* ids = (int*)(ws + o_ids);
    int* tids = (int*)(ws + o_tids);
    int* ntied = (int*)(ws + o_nt);
    unsigned long long* k1 = (unsigned long long*)(ws + o_k1);
    unsigned long long* k2 = (unsigned long long*)(ws + o_k2);
    int* r1 = (int*)(ws + o_r1);
    int* r2 = (int*)(ws + o_r2);
    unsigned long long* skeys = (unsigned long long*)(ws + o_sk);
    int* sstart = (int*)(ws + o_ss);
    unsigned long long* tkeys = (unsigned long long*)(ws + o_tk);
    unsigned long long* akeys = (unsigned long long*)(ws + o_ak);
    int* astart = (int*)(ws + o_as);
    const int rbits = bits_for(k);
    int hnt = 0;
    hipLaunchKernelGGL(k_wreg_scan, dim3(gn), dim3(256), 0, s, n, k, t->dist, t->delta, t->region, tied);
    hipError_t e = hipGetLastError();
    // the tied nodes in ascending id order
    if (e == hipSuccess) {
        size_t tb = 0;
        hipcub::CountingInputIterator<int> iota(0);
        e = hipcub::DeviceSelect::Flagged(nullptr, tb, iota, tied, ids, ntied, n, s);
        void* tmp = nullptr;
        if (e == hipSuccess && salloc(&tmp, std::max<size_t>(tb, 1)) != SSM_OK) e = hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipcub::DeviceSelect::Flagged(tmp, tb, iota, tied, ids, ntied, n, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hnt, ntied, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipStreamSynchronize(s);
        if (tmp) sfree(tmp);
    }
    // the single nodes' deltas sorted by (region, delta): by delta, then
    // stably by region; tied nodes carry region k and land past the regions
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wreg_keys, dim3(gn), dim3(256), 0, s, n, k, t->delta, t->region, true, k1, r1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = sort_pairs(k1, k2, r1, r2, n, 64, s);
    if (e == hipSuccess) e = sort_pairs(r2, r1, k2, skeys, n, rbits, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wreg_starts, dim3(std::min(div_up(n + 1, 256), 4096)), dim3(256), 0, s, n, k, r1, sstart);
        e = hipGetLastError();
    }
    // tied nodes by (delta, id), then resolved level by level
    if (e == hipSuccess && hnt > 0) {
        hipLaunchKernelGGL(k_gather_dkeys, dim3(std::min(div_up(hnt, 256), 4096)), dim3(256), 0, s, hnt, ids,
                           t->delta, k1);
        e = hipGetLastError();
        if (e == hipSuccess) e = sort_pairs(k1, tkeys, ids, tids, hnt, 64, s);
        if (e == hipSuccess) {
            const size_t lds = sizeof(int) * (size_t)k;
            if (lds > 64 * 1024)
                (void)hipFuncSetAttribute((const void*)k_wreg_ties, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds);
            hipLaunchKernelGGL(k_wreg_ties, dim3(1), dim3(1024), lds, s, n, k, hnt, tids, tkeys, t->dist, skeys,
                               sstart, t->region);
            e = hipGetLastError();
        }
    }
    // every member's delta sorted by (region, delta) for the counts s
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wreg_keys, dim3(gn), dim3(256), 0, s, n, k, t->delta, t->region, false, k1, r1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = sort_pairs(k1, k2, r1, r2, n, 64, s);
    if (e == hipSuccess) e = sort_pairs(r2, r1, k2, akeys, n, rbits, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wreg_starts, dim3(std::min(div_up(n + 1, 256), 4096)), dim3(256), 0, s, n, k, r1, astart);
        const long long total = (long long)k * n;
        hipLaunchKernelGGL(k_wterms, dim3(std::min(div_up(total, 256), 16384)), dim3(256), 0, s, n, k, g->row_ptr,
                           g->col_idx, t->pivots, t->dist, akeys, astart, t->w64, t->wd32);
        hipLaunchKernelGGL(k_wden, dim3(gn), dim3(256), 0, s, n, k, g->row_ptr, len, t->w64, t->den64, t->den32,
                           t->wl32);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    sfree(ws);
    return e == hipSuccess ? SSM_OK : hip_fail(e, "regions and terms (edge lengths)");
}

}  // namespace ssm

using namespace ssm;

extern "C" {

void ssm_wterms_free(ssm_wterms* t) {
    if (!t) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    (void)hipDeviceSynchronize();  // the scratch cache takes the arena back once the device is idle
    sfree(t->arena);               // every buffer of the handle
    (void)hipSetDevice(cur);
    delete t;
}

ssm_status ssm_select_pivots_w(const ssm_csr* g, const double* len, int32_t k, int32_t first, int32_t* pivots,
                               double* dist, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!len || !pivots) return fail(SSM_E_INVAL, "NULL lengths or pivots");
    if (k < 1 || k > g->n) return fail(SSM_E_INVAL, "k must lie in [1, n]");
    if (first < 0 || first >= g->n) return fail(SSM_E_INVAL, "first must lie in [0, n)");
    if ((long long)k * g->n >= (1LL << 40)) return fail(SSM_E_RANGE, "k * n too large");
    st = select_pivots_w(g, len, k, first, pivots, stream);
    if (st != SSM_OK || !dist) return st;
    return sssp_rows(g, len, k, pivots, dist, stream);
}

ssm_status ssm_sssp_pivots(const ssm_csr* g, const double* len, int32_t k, const int32_t* pivots, double* dist,
                           hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!len || !pivots || !dist) return fail(SSM_E_INVAL, "NULL argument");
    if (k < 1 || k > g->n) return fail(SSM_E_INVAL, "k must lie in [1, n]");
    if ((long long)k * g->n >= (1LL << 40)) return fail(SSM_E_RANGE, "k * n too large");
    return sssp_rows(g, len, k, pivots, dist, stream);
}

ssm_status ssm_build_terms_w(const ssm_csr* g, const double* len, int32_t k, const int32_t* pivots,
                             const double* dist, ssm_wterms** out, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!len || !pivots || !dist || !out) return fail(SSM_E_INVAL, "NULL argument");
    if (k < 1 || k > g->n) return fail(SSM_E_INVAL, "k must lie in [1, n]");
    const int n = g->n;
    ssm_wterms* t = new ssm_wterms();
    (void)hipGetDevice(&t->device);
    t->n = n;
    t->k = k;
    t->nnz = g->nnz;
    const size_t kn = (size_t)k * n;
    struct {
        void** p;
        size_t bytes;
    } allocs[] = {
        {(void**)&t->pivots, sizeof(int) * (size_t)k}, {(void**)&t->dist, sizeof(double) * kn},
        {(void**)&t->delta, sizeof(double) * n},       {(void**)&t->region, sizeof(int) * n},
        {(void**)&t->w64, sizeof(double) * kn},        {(void**)&t->wd32, sizeof(float2) * kn},
        {(void**)&t->den64, sizeof(double) * n},       {(void**)&t->den32, sizeof(float) * n},
        {(void**)&t->wl32, sizeof(float2) * (size_t)std::max(g->nnz, 1)},
        {(void**)&t->xtmp, sizeof(double) * 2 * (size_t)n},
    };
    // one allocation, carved at 256-byte boundaries, from the scratch cache
    // (every buffer is written before it is read)
    size_t total = 0;
    for (auto& a : allocs) total += (a.bytes + 255) / 256 * 256;
    st = salloc(&t->arena, total);
    if (st != SSM_OK) {
        ssm_wterms_free(t);
        return st;
    }
    size_t off = 0;
    for (auto& a : allocs) {
        *a.p = (char*)t->arena + off;
        off += (a.bytes + 255) / 256 * 256;
    }
    hipError_t e = hipMemcpyAsync(t->pivots, pivots, sizeof(int) * (size_t)k, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t->dist, dist, sizeof(double) * kn, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) {
        ssm_wterms_free(t);
        return hip_fail(e, "terms (edge lengths): copy");
    }
    st = build_wterms(g, len, t, stream);
    if (st != SSM_OK) {
        ssm_wterms_free(t);
        return st;
    }
    *out = t;
    return SSM_OK;
}

ssm_status ssm_wterms_export(const ssm_wterms* t, double* delta_host, int32_t* region_host, double* w_host,
                             double* den_host) {
    if (!t) return fail(SSM_E_INVAL, "NULL terms");
    const size_t n = t->n, kn = (size_t)t->k * t->n;
    if (delta_host) SSM_HIP(hipMemcpy(delta_host, t->delta, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (region_host) SSM_HIP(hipMemcpy(region_host, t->region, sizeof(int) * n, hipMemcpyDeviceToHost));
    if (w_host) SSM_HIP(hipMemcpy(w_host, t->w64, sizeof(double) * kn, hipMemcpyDeviceToHost));
    if (den_host) SSM_HIP(hipMemcpy(den_host, t->den64, sizeof(double) * n, hipMemcpyDeviceToHost));
    return SSM_OK;
}

ssm_status ssm_pivotmds_init_w(const ssm_csr* g, const double* len, const ssm_wterms* t, ssm_prec p, void* x,
                               hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!len || !t || !x) return fail(SSM_E_INVAL, "NULL argument");
    if (t->n != g->n) return fail(SSM_E_INVAL, "terms were built for another graph");
    if (t->k < 3) return fail(SSM_E_INVAL, "PivotMDS needs k >= 3");
    if (p != SSM_FP64 && p != SSM_FP32) return fail(SSM_E_INVAL, "unknown precision");
    return pivotmds_w(g, len, t->k, t->dist, p, x, stream);
}

ssm_status ssm_majorize_w(const ssm_csr* g, const double* len, ssm_wterms* t, ssm_prec p, void* x, int32_t iters,
                          hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!len || !t || !x) return fail(SSM_E_INVAL, "NULL argument");
    if (t->n != g->n) return fail(SSM_E_INVAL, "terms were built for another graph");
    if (iters < 0) return fail(SSM_E_INVAL, "iters < 0");
    if (p != SSM_FP64 && p != SSM_FP32) return fail(SSM_E_INVAL, "unknown precision");
    const int n = g->n, k = t->k;
    const int grid = std::max(1, std::min(div_up(n, 256), num_cus() * 8));
    const int grid32 = std::max(1, std::min(div_up(n, 64), num_cus() * 8));
    void* a = x;
    void* b = t->xtmp;
    for (int it = 0; it < iters; ++it) {
        if (p == SSM_FP64)
            hipLaunchKernelGGL(k_wsweep_f64, dim3(grid), dim3(256), sizeof(double2) * (size_t)k, stream, n, k,
                               g->row_ptr, g->col_idx, len, (const double2*)a, (double2*)b, t->pivots, t->dist,
                               t->w64, t->den64);
        else
            hipLaunchKernelGGL(k_wsweep_f32, dim3(grid32), dim3(64 * kWSplit),
                               sizeof(float2) * ((size_t)k + 64 * kWSplit), stream, n, k, g->row_ptr, g->col_idx,
                               t->wl32, (const float2*)a, (float2*)b, t->pivots, t->wd32, t->den32);
        void* c = a;
        a = b;
        b = c;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && a != x)
        e = hipMemcpyAsync(x, a, (p == SSM_FP64 ? sizeof(double2) : sizeof(float2)) * (size_t)n,
                           hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "sweeps (edge lengths)");
    return SSM_OK;
}

ssm_status ssm_majorize_mixed_w(const ssm_csr* g, const double* len, ssm_wterms* t, double* x64, float* x32,
                                int32_t iters, int32_t warm, hipStream_t stream) {
    if (!x64 || !x32) return fail(SSM_E_INVAL, "NULL layout");
    if (warm < 1) return fail(SSM_E_INVAL, "warm must be >= 1");
    const int w = std::min(warm, iters);
    ssm_status st = ssm_majorize_w(g, len, t, SSM_FP64, x64, w, stream);
    if (st != SSM_OK) return st;
    hipLaunchKernelGGL(k_wround, dim3(std::max(1, std::min(div_up(g->n, 256), 8192))), dim3(256), 0, stream, g->n,
                       (const double2*)x64, (float2*)x32);
    SSM_HIP(hipGetLastError());
    return ssm_majorize_w(g, len, t, SSM_FP32, x32, iters - w, stream);
}

ssm_status ssm_stress_w(const ssm_csr* g, const double* len, const ssm_wterms* t, ssm_prec p, const void* x,
                        double* out_host, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!len || !t || !x || !out_host) return fail(SSM_E_INVAL, "NULL argument");
    if (t->n != g->n) return fail(SSM_E_INVAL, "terms were built for another graph");
    if (p != SSM_FP64 && p != SSM_FP32) return fail(SSM_E_INVAL, "unknown precision");
    const int n = g->n, k = t->k;
    const int nb = std::max(1, std::min(div_up(n, 256), 2048));
    double* ws = nullptr;
    st = salloc((void**)&ws, sizeof(double) * ((size_t)nb + 1));
    if (st != SSM_OK) return st;
    if (p == SSM_FP64)
        hipLaunchKernelGGL(k_wstress<double2>, dim3(nb), dim3(256), 0, stream, n, k, g->row_ptr, g->col_idx, len,
                           (const double2*)x, t->pivots, t->dist, t->w64, ws);
    else
        hipLaunchKernelGGL(k_wstress<float2>, dim3(nb), dim3(256), 0, stream, n, k, g->row_ptr, g->col_idx, len,
                           (const float2*)x, t->pivots, t->dist, t->w64, ws);
    launch_sum_partials(ws, nb, ws + nb, stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, ws + nb, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipStreamSynchronize(stream);
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "stress (edge lengths)");
    return SSM_OK;
}

}  // extern "C"
