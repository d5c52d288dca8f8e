// Layout pool: many small graphs laid out together (Algorithm 1 per graph,
// batched across graphs).  Each graph keeps its CSR, distance words, weight
// tables and coordinates resident in one device arena; every stage runs for
// a whole list of graphs per launch:
//   - selection, BFS, regions/terms, PivotMDS statistics and eigen step:
//     one workgroup per graph (or per (graph, rank) / (graph, chunk) item);
//   - sweeps: one launch per sweep over the 64-node chunks of every listed
//     graph (one wavefront per chunk), so a graph of 2,000 nodes costs 32
//     waves of a launch rather than a launch of its own.
// The arithmetic of every step is the single-graph path's: the same rule R1
// regions, adapted weights and denominators (Section 3), PivotMDS with the
// same eigen solver, the FP64 sweep in the oracle's operation order, and the
// FP32 displacement form of Eq. 5.
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "change.h"
#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

// ------------------------------------------------------------- kernels

// One workgroup per graph: delta and the candidate count per node, regions
// by rule R1 level by level (single candidates join first, tied nodes then
// pick the smallest (size snapshot, rank)), the cumulative histograms H, the
// weight tables w64 / wt2, the denominators and the packed distances.
__global__ __launch_bounds__(1024) void k_pool_regions(const PoolGraph* __restrict__ gs) {
#pragma clang fp contract(off)
    extern __shared__ int psh[];
    const PoolGraph& g = gs[blockIdx.x];
    const int n = g.n, k = g.k, kpad = g.kpad, W = g.W;
    const int* __restrict__ dist = g.dist;
    int* size = psh;                                               // [k]
    int* snap = size + k;                                          // [k]
    unsigned* tied = (unsigned*)(snap + k);                        // [(n + 31) / 32]
    unsigned short* dl = (unsigned short*)(tied + (n + 31) / 32);  // [n] delta
    __shared__ int red[1024 / kWave];
    for (int t = threadIdx.x; t < k; t += blockDim.x) size[t] = 0;
    for (int w = threadIdx.x; w < (n + 31) / 32; w += blockDim.x) tied[w] = 0u;
    __syncthreads();
    int dm = 0;
    constexpr int U = 8;  // distance loads in flight per thread
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int best = INT_MAX, cnt = 0, at = 0;
        for (int t0 = 0; t0 < k; t0 += U) {
            int dv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) dv[j] = t0 + j < k ? dist[(size_t)(t0 + j) * n + i] : INT_MAX;
#pragma unroll
            for (int j = 0; j < U; ++j) {  // ranks in ascending order
                if (t0 + j >= k) break;
                const int d = dv[j];
                if (d < best) {
                    best = d;
                    cnt = 1;
                    at = t0 + j;
                } else if (d == best) {
                    ++cnt;
                }
            }
        }
        g.delta[i] = best;
        dl[i] = (unsigned short)best;
        g.region[i] = cnt == 1 ? at : -1;
        if (cnt > 1) atomicOr(&tied[i >> 5], 1u << (i & 31));
        dm = max(dm, best);
    }
    const int delta_max = block_max(dm, red);
    // each node i is visited by the same thread in every pass below
    for (int l = 0; l <= delta_max; ++l) {
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if (dl[i] == l && !((tied[i >> 5] >> (i & 31)) & 1u)) atomicAdd(&size[g.region[i]], 1);
        __syncthreads();
        for (int t = threadIdx.x; t < k; t += blockDim.x) snap[t] = size[t];
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (dl[i] != l || !((tied[i >> 5] >> (i & 31)) & 1u)) continue;
            int pick = -1;
            for (int t0 = 0; t0 < k; t0 += U) {
                int dv[U];
#pragma unroll
                for (int j = 0; j < U; ++j) dv[j] = t0 + j < k ? dist[(size_t)(t0 + j) * n + i] : -1;
#pragma unroll
                for (int j = 0; j < U; ++j) {  // ranks in ascending order
                    const int t = t0 + j;
                    if (dv[j] != l) continue;
                    if (pick < 0 || snap[t] < snap[pick]) pick = t;
                }
            }
            g.region[i] = pick;
            atomicAdd(&size[pick], 1);
        }
        __syncthreads();
    }
    // raw histogram of (region, delta) by device atomics, read back by
    // device-scope loads (no stale line of the zeroed table can be used)
    const int L = delta_max + 1;
    for (int q = threadIdx.x; q < k * L; q += blockDim.x) g.H[q] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&g.H[(size_t)g.region[i] * L + dl[i]], 1);
    __syncthreads();
    // per rank: running sum over the level and the weight row in one walk
    // (the level needed for distance d is min(d / 2, delta_max), which never
    // decreases with d)
    for (int d = threadIdx.x; d < W; d += blockDim.x)
        g.invd[d] = d >= 2 ? make_float2((float)(1.0 / ((double)d * (double)d)), (float)(1.0 / (double)d))
                           : make_float2(0.f, 0.f);
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) {
        if (t >= k) {
            for (int d = 0; d < W; ++d) {
                g.w64[(size_t)t * W + d] = 0.0;
                g.wt2[(size_t)t * W + d] = make_float2(0.f, 0.f);
            }
            for (int l = 0; l < L; ++l) g.Hf[(size_t)t * L + l] = 0.f;
            g.pivots[t] = g.pivots[0];
            continue;
        }
        int acc = 0, l = -1;
        for (int d = 0; d < W; ++d) {
            const int half = min(d / 2, L - 1);
            while (l < half) {
                ++l;
                acc += __hip_atomic_load(&g.H[(size_t)t * L + l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                g.H[(size_t)t * L + l] = acc;
                g.Hf[(size_t)t * L + l] = (float)acc;
            }
            const double val = d >= 2 ? (double)acc / (double)((long long)d * (long long)d) : 0.0;
            g.w64[(size_t)t * W + d] = val;
            g.wt2[(size_t)t * W + d] = make_float2((float)val, (float)(val * (double)d));
        }
        while (l < L - 1) {
            ++l;
            acc += __hip_atomic_load(&g.H[(size_t)t * L + l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            g.H[(size_t)t * L + l] = acc;
            g.Hf[(size_t)t * L + l] = (float)acc;
        }
    }
    __syncthreads();
    // den_i = deg(i) + sum over ranks ascending of w'_it (d >= 2)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double s = 0.0;
        for (int e = g.rp[i]; e < g.rp[i + 1]; ++e) s += 1.0;
        for (int t0 = 0; t0 < k; t0 += U) {
            int dv[U];
            double wv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) dv[j] = t0 + j < k ? dist[(size_t)(t0 + j) * n + i] : 0;
#pragma unroll
            for (int j = 0; j < U; ++j) wv[j] = dv[j] >= 2 ? g.w64[(size_t)(t0 + j) * W + dv[j]] : 0.0;
#pragma unroll
            for (int j = 0; j < U; ++j)  // ranks in ascending order
                if (dv[j] >= 2) s += wv[j];
        }
        g.den64[i] = s;
        g.den32[i] = (float)s;
    }
    // packed words, four per thread and pass: every load of a pass before
    // its stores
    const long long words = (long long)(kpad / 8) * n;
    constexpr int QW = 4;
    for (long long q0 = threadIdx.x; q0 < words; q0 += QW * (long long)blockDim.x) {
        int dv[QW][8];
#pragma unroll
        for (int w = 0; w < QW; ++w) {
            const long long q = q0 + (long long)w * blockDim.x;
            const int b = (int)(q / n), i = (int)(q % n);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int t = b * 8 + j;
                dv[w][j] = q < words && t < k ? dist[(size_t)t * n + i] : 0;
            }
        }
#pragma unroll
        for (int w = 0; w < QW; ++w) {
            const long long q = q0 + (long long)w * blockDim.x;
            if (q >= words) break;
            union {
                uint4 v;
                uint16_t e[8];
            } u;
#pragma unroll
            for (int j = 0; j < 8; ++j) u.e[j] = (uint16_t)dv[w][j];
            g.dpk[q] = u.v;
        }
    }
    if (threadIdx.x == 0) g.info[2] = delta_max;
}

// FP64 sweep, one thread per node, items (graph, first node of 256): Eq. 5
// in the oracle's order (neighbours at a positive distance in CSR order,
// then the zero-distance votes, then pivot terms by ascending rank), from
// x64[src] into x64[src ^ 1].
__global__ __launch_bounds__(256) void k_pool_sweep64(const PoolGraph* __restrict__ gs,
                                                      const int2* __restrict__ items, int src) {
#pragma clang fp contract(off)
    const int2 st = items[blockIdx.x];
    const PoolGraph& g = gs[st.x];
    const int n = g.n, W = g.W, nwords = g.kpad / 8;
    const int i = st.y + threadIdx.x;
    if (i >= n) return;
    const double2* __restrict__ xo = g.x64[src];
    double2* __restrict__ xn = g.x64[src ^ 1];
    const double2 xv = xo[i];
    const double xi = xv.x, yi = xv.y;
    double nx = 0.0, ny = 0.0;
    int zero = 0;
    for (int e = g.rp[i]; e < g.rp[i + 1]; ++e) {
        const double2 xj = xo[g.ci[e]];
        double dx = xi - xj.x, dy = yi - xj.y;
        double r = sqrt(dx * dx + dy * dy);
        if (r > 0.0) {
            nx += xj.x + dx / r;
            ny += xj.y + dy / r;
        } else {
            ++zero;
        }
    }
    for (int z = 0; z < zero; ++z) {
        nx += xi;
        ny += yi;
    }
    for (int b = 0; b < nwords; ++b) {
        union {
            uint4 v;
            uint16_t e[8];
        } u;
        u.v = g.dpk[(size_t)b * n + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int d = (int)u.e[j];
            if (d < 2) continue;
            const int t = b * 8 + j;
            const double w = g.w64[(size_t)t * W + d];
            const double2 p = xo[g.pivots[t]];
            double dx = xi - p.x, dy = yi - p.y;
            double r = sqrt(dx * dx + dy * dy);
            double vx = p.x, vy = p.y;
            if (r > 0.0) {
                vx = p.x + (double)d * dx / r;
                vy = p.y + (double)d * dy / r;
            }
            nx += w * vx;
            ny += w * vy;
        }
    }
    const double dn = g.den64[i];
    xn[i] = make_double2(nx / dn, ny / dn);
}

// x32[0] = x64[src] rounded to FP32.
__global__ __launch_bounds__(256) void k_pool_round(const PoolGraph* __restrict__ gs,
                                                    const int2* __restrict__ items, int src) {
    const int2 st = items[blockIdx.x];
    const PoolGraph& g = gs[st.x];
    const int i = st.y + threadIdx.x;
    if (i >= g.n) return;
    const double2 v = g.x64[src][i];
    g.x32[0][i] = make_float2((float)v.x, (float)v.y);
}

constexpr int kPoolSweepBlock = 256;     // nodes of one graph per block
constexpr int kPoolHistLds = 40 * 1024;  // LDS for a graph's Hf and invd tables in the FP32 sweep

// Whether the FP32 sweep of a graph stages its region histograms and 1/d
// table in LDS (decided per graph, so a graph's arithmetic never depends on
// the graphs that share its launch).
inline int pool_hist_mode(int kpad, int L, int W) {
    return sizeof(float) * (size_t)kpad * L + sizeof(float2) * (size_t)W <= (size_t)kPoolHistLds;
}

// FP32 sweep s of a call on one 256-node chunk ch = (graph, first node) of
// one graph, by a block of 256 threads (thread = node).  A graph takes part
// while s < its iters; it reads x32[(parity + s) & 1] and writes the other
// buffer.  Eq. 5 in displacement form as the single-graph FP32 sweep:
// neighbours in CSR order first, then pivot terms by ascending rank with
// f = w' - (w' d) / r, where w' = H[t][min(d/2, delta_max)] / d^2 comes from
// the LDS copies of Hf and (1/d^2, 1/d) when the graph's tables fit (else from
// the (w', w' d) table in global memory).  Pivot coordinates are staged in
// LDS for the chunk.  Uniform exits come before the staging barrier.
__device__ __forceinline__ void pool_sweep_chunk(const PoolGraph* __restrict__ gs, int2 ch, int s, float4* psm) {
    const PoolGraph& g = gs[ch.x];
    if (s >= g.iters) return;  // the whole block
    const int n = g.n, W = g.W, L = g.L, kpad = g.kpad, nwords = kpad / 8;
    const bool hist = g.hist != 0;
    const int p = (g.parity + s) & 1;
    const float2* __restrict__ xo = g.x32[p];
    float2* __restrict__ xn = g.x32[p ^ 1];
    if (g.tol > 0.0 && g.info[6]) {  // the graph met its stop test: carry its iterate over
        const int i = ch.y + threadIdx.x;
        if (i < n) xn[i] = xo[i];
        return;  // the whole block
    }
    float2* sP = (float2*)psm;                   // [kpad]
    float2* sInv = sP + kpad;                    // [W] (hist)
    float* sH = (float*)(sInv + (hist ? W : 0));  // [kpad][L] (hist)
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) sP[t] = xo[g.pivots[t]];
    if (hist) {
        for (int d = threadIdx.x; d < W; d += blockDim.x) sInv[d] = g.invd[d];
        for (int q = threadIdx.x; q < kpad * L; q += blockDim.x) sH[q] = g.Hf[q];
    }
    __syncthreads();
    const int i = ch.y + threadIdx.x;
    if (i >= n) return;
    const float tiny = 1e-30f;
    const float2 xi = xo[i];
    float ax = 0.f, ay = 0.f;
    const int e0 = g.rp[i], e1 = g.rp[i + 1];
    for (int e = e0; e < e1; e += 4) {
        int j[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cj = g.ci[min(e + q, e1 - 1)];  // unconditional load
            j[q] = e + q < e1 ? cj : i;               // a missing slot reads x_i: adds exactly 0
        }
        float2 xj[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) xj[q] = xo[j[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float dx = xj[q].x - xi.x, dy = xj[q].y - xi.y;
            const float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
            const float f = 1.f - inv;  // w = 1, d = 1
            ax += f * dx;
            ay += f * dy;
        }
    }
    const uint4* __restrict__ dp = g.dpk + i;
    uint4 wa = nwords > 0 ? dp[0] : make_uint4(0, 0, 0, 0);
    uint4 wb = nwords > 1 ? dp[(size_t)n] : make_uint4(0, 0, 0, 0);
    for (int b = 0; b < nwords; ++b) {
        union {
            uint4 v;
            uint16_t e[8];
        } u;
        u.v = wa;
        wa = wb;
        if (b + 2 < nwords) wb = dp[(size_t)(b + 2) * n];  // two words ahead
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int t = b * 8 + jj;
            const int d = (int)u.e[jj];
            const float2 pv = sP[t];
            const float dx = pv.x - xi.x, dy = pv.y - xi.y;
            const float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
            float f;
            if (hist) {
                const float h = sH[t * L + min(d >> 1, L - 1)];
                const float2 id = sInv[d];
                f = fmaf(-id.y, inv, id.x) * h;
            } else {
                const float2 f01 = g.wt2[(size_t)t * W + d];
                f = fmaf(-f01.y, inv, f01.x);
            }
            ax += f * dx;
            ay += f * dy;
        }
    }
    const float dn = g.den32[i];
    xn[i] = make_float2(xi.x + ax / dn, xi.y + ay / dn);
}

// The pooled FP32 sweep s over the staged chunk list (hdr[0] chunks).
// PERSIST = false: block b takes chunk b (the grid may be rounded up for a
// reusable graph; the extra blocks return).  PERSIST = true: a grid sized to
// the device (blocks resident at once) loops over the chunks, restaging LDS
// per chunk.  A node's arithmetic is the same either way, bit for bit.
template <bool PERSIST>
__global__ __launch_bounds__(kPoolSweepBlock) void k_pool_sweep32(const PoolGraph* __restrict__ gs,
                                                                  const int2* __restrict__ chunks,
                                                                  const int* __restrict__ hdr, int s) {
    extern __shared__ float4 psm[];
    const int nch = hdr[0];
    if (!PERSIST) {
        if ((int)blockIdx.x < nch) pool_sweep_chunk(gs, chunks[blockIdx.x], s, psm);
        return;
    }
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {  // uniform over the block
        __syncthreads();  // the previous chunk's LDS reads are done
        pool_sweep_chunk(gs, chunks[c], s, psm);
    }
}

// Algorithm 1's stop test after pool sweep s (change.h): the twelve moments
// of each listed 256-node chunk of a graph that has a tolerance and has not
// stopped yet, relative to o = the graph's node 0 in the old iterate.
__global__ __launch_bounds__(256) void k_pool_moments(const PoolGraph* __restrict__ gs, const int2* __restrict__ chunks,
                                                      const int* __restrict__ hdr, int s,
                                                      double* __restrict__ partial) {
    if ((int)blockIdx.x >= hdr[0]) return;  // a grid rounded up for a reusable graph
    const int2 ch = chunks[blockIdx.x];
    const PoolGraph& g = gs[ch.x];
    if (s >= g.iters || !(g.tol > 0.0) || g.info[6]) return;  // the whole block
    const int p = (g.parity + s) & 1;
    const float2* __restrict__ xo = g.x32[p];
    const float2* __restrict__ xn = g.x32[p ^ 1];
    const double2 o = to_d2(xo[0]);
    double m[kMoments];
#pragma unroll
    for (int j = 0; j < kMoments; ++j) m[j] = 0.0;
    const int i = ch.y + threadIdx.x;
    if (i < g.n) moments_add(m, o, to_d2(xo[i]), to_d2(xn[i]));
    __shared__ double red[(256 / kWave) * kMoments];
    const double v = block_moments(m, red);
    if (threadIdx.x < kMoments) partial[(size_t)blockIdx.x * kMoments + threadIdx.x] = v;
}

// One wave per listed graph: lane l sums the chunk partials first[q] + l,
// + l + 64, ... in order, a fixed-order wave sum adds the lanes' (the same
// order whatever else the batch holds); a change <= tol after sweep s sets
// info[6] and records the sweeps run in info[7].
__global__ __launch_bounds__(256) void k_pool_decide(const PoolGraph* __restrict__ gs, const int* __restrict__ hdr,
                                                     const int* __restrict__ first,
                                                     const double* __restrict__ partial, int s) {
    const int q = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (q >= hdr[1]) return;  // the whole wave
    const PoolGraph& g = gs[q];
    if (s >= g.iters || !(g.tol > 0.0) || g.info[6]) return;  // the whole wave
    double m[kMoments];
#pragma unroll
    for (int j = 0; j < kMoments; ++j) m[j] = 0.0;
    for (int c = first[q] + lane_id(); c < first[q + 1]; c += kWave)
#pragma unroll
        for (int j = 0; j < kMoments; ++j) m[j] += partial[(size_t)c * kMoments + j];
#pragma unroll
    for (int j = 0; j < kMoments; ++j) m[j] = wave_sum_dpp(m[j]);
    if (lane_id() == 0 && rigid_change(m, g.n) <= g.tol) {
        g.info[7] = g.done0 + s + 1;
        g.info[6] = 1;
    }
}

// Sparse stress s' (Eq. 3) in FP64 of each graph's current FP32 iterate
// x32[parity]: one wavefront per 64-node chunk writes its share to
// partial[chunk] (edge terms i < j over the chunk's arcs, then the pivot
// terms of its nodes).
__global__ __launch_bounds__(256) void k_pool_stress(const PoolGraph* __restrict__ gs, const int2* __restrict__ chunks,
                                                     int nchunks, double* __restrict__ partial) {
    const int c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (c >= nchunks) return;  // whole wave
    const int2 ch = chunks[c];
    const PoolGraph& g = gs[ch.x];
    const int n = g.n, W = g.W, nwords = g.kpad / 8;
    const float2* __restrict__ x = g.x32[g.parity];
    double acc = 0.0;
    wave_arcs(n, g.rp, g.ci, ch.y, [&](int i, int j) {
        if (j <= i) return;
        const float2 a = x[i], b = x[j];
        const double dx = (double)a.x - (double)b.x, dy = (double)a.y - (double)b.y;
        const double r = sqrt(dx * dx + dy * dy);
        acc += (r - 1.0) * (r - 1.0);
    });
    const int i = ch.y + lane_id();
    if (i < n) {
        const float2 a = x[i];
        for (int b = 0; b < nwords; ++b) {
            union {
                uint4 v;
                uint16_t e[8];
            } u;
            u.v = g.dpk[(size_t)b * n + i];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int d = (int)u.e[j];
                if (d < 2) continue;
                const int t = b * 8 + j;
                const float2 pv = x[g.pivots[t]];
                const double dx = (double)a.x - (double)pv.x, dy = (double)a.y - (double)pv.y;
                const double r = sqrt(dx * dx + dy * dy);
                acc += g.w64[(size_t)t * W + d] * (r - d) * (r - d);
            }
        }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) partial[c] = acc;
}

// out[q] = sum of partial[first[q] .. first[q + 1]) in ascending order.
__global__ void k_pool_stress_sum(int count, const int* __restrict__ first, const double* __restrict__ partial,
                                  double* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    double s = 0.0;
    for (int c = first[q]; c < first[q + 1]; ++c) s += partial[c];
    out[q] = s;
}

// Items (graph, first row of 256): info[5] = 1 if a row has a self-loop, a
// repeated neighbour or an arc whose reverse is missing (linear scans: the
// pool's graphs have small degrees).
__global__ __launch_bounds__(256) void k_pool_validate(const PoolGraph* __restrict__ gs,
                                                       const int2* __restrict__ items) {
    const int2 st = items[blockIdx.x];
    const PoolGraph& g = gs[st.x];
    const int i = st.y + threadIdx.x;
    if (i >= g.n) return;
    const int e0 = g.rp[i], e1 = g.rp[i + 1];
    bool bad = false;
    for (int e = e0; e < e1 && !bad; ++e) {
        const int j = g.ci[e];
        if (j == i) bad = true;
        for (int f = e0; f < e && !bad; ++f) bad = g.ci[f] == j;
        bool back = false;
        for (int f = g.rp[j]; f < g.rp[j + 1] && !back; ++f) back = g.ci[f] == i;
        bad = bad || !back;
    }
    if (bad) atomicOr(&g.info[5], 1);
}

// info words of each listed graph into one array (for a single copy back).
__global__ void k_pool_gather_info(const PoolGraph* __restrict__ gs, int count, int* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count * 8) return;
    out[q] = gs[q / 8].info[q % 8];
}

// --------------------------------------------------------------- arena

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kNone = ~(size_t)0;

size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over one device allocation; free ranges are kept by
// offset and merged with their neighbours on release.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    std::map<size_t, size_t> free_;

    size_t alloc(size_t bytes) {
        bytes = align_up(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rem = it->second - bytes;
            free_.erase(it);
            if (rem) free_[off + bytes] = rem;
            used += bytes;
            return off;
        }
        return kNone;
    }
    void release(size_t off, size_t bytes) {
        if (off == kNone) return;
        bytes = align_up(std::max<size_t>(bytes, 1));
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Bump layout of one arena block: offsets of consecutive aligned arrays.
struct Layout {
    size_t bytes = 0;
    size_t add(size_t b) {
        const size_t o = bytes;
        bytes += align_up(b);
        return o;
    }
};

enum SlotState { kFree = 0, kAdded = 1, kReady = 2, kFailed = 3 };

struct Slot {
    int state = kFree;
    int n = 0, nnz = 0, k = 0, kpad = 0, first = 0, target = 0, done = 0, parity = 0;
    int dmax = 0, delta_max = 0, fail = 0, x64cur = 0;
    double tol = 0.0;  // stop test of the FP32 sweeps (0: a fixed sweep count)
    size_t off_p = kNone, sz_p = 0, off_s = kNone, sz_s = 0, off_t = kNone, sz_t = 0;
    PoolGraph g{};
};

// Staging of one asynchronous sweep call: host copies and device buffer
// stay untouched until `done` has fired.
// A captured sweep quantum: the launches of `most` sweeps (and stop tests)
// over grids rounded up to (chunks, graphs), with LDS `lds`; the kernels take
// the real counts from the stage header, so one graph serves every call whose
// counts round to the same buckets.
struct QuantumKey {
    int chunks, graphs, most, lds, tol, persist;
    bool operator<(const QuantumKey& o) const {
        if (chunks != o.chunks) return chunks < o.chunks;
        if (graphs != o.graphs) return graphs < o.graphs;
        if (most != o.most) return most < o.most;
        if (lds != o.lds) return lds < o.lds;
        if (tol != o.tol) return tol < o.tol;
        return persist < o.persist;
    }
};

// Shape class of a pooled sweep for its schedule choice: rounded chunk and
// graph counts and the LDS bytes.
struct ScheduleKey {
    int chunks, graphs, lds;
    bool operator<(const ScheduleKey& o) const {
        if (chunks != o.chunks) return chunks < o.chunks;
        if (graphs != o.graphs) return graphs < o.graphs;
        return lds < o.lds;
    }
};

struct Stage {
    std::vector<PoolGraph> hg;
    std::vector<int2> hc;
    char* dev = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    std::map<QuantumKey, hipGraphExec_t> graphs;  // captured quanta over dev's layout
};

}  // namespace

}  // namespace ssm

struct ssm_pool {
    int device = 0;
    ssm::Arena arena;
    std::vector<ssm::Slot> slots;
    std::vector<int> free_ids;
    int2* tiles = nullptr;  // Gram tile list for up to kPoolMaxK / 16 tile columns
    ssm::Stage stage[2];
    int flip = 0;
    hipStream_t capture = nullptr;  // where sweep quanta are captured (never run on)
    bool no_graphs = false;         // capture failed once: launch directly
    std::map<ssm::ScheduleKey, int> schedule;  // timed choice: 1 = persistent grid, 0 = a block per chunk
    std::mutex mu;  // calls on one pool are serialized
};

namespace ssm {
namespace {

int tile_cols(int k) { return (k + 15) / 16; }

ssm_status wait_stage(Stage& st) {
    if (st.pending) {
        hipError_t e = hipEventSynchronize(st.done);
        st.pending = false;
        if (e != hipSuccess) return hip_fail(e, "pool: wait for a previous sweep");
    }
    return SSM_OK;
}

ssm_status wait_all(ssm_pool* p) {
    for (auto& st : p->stage) {
        ssm_status r = wait_stage(st);
        if (r != SSM_OK) return r;
    }
    return SSM_OK;
}

// Fills the device pointers of slot s from its blocks.
void bind(ssm_pool* p, Slot& s) {
    PoolGraph& g = s.g;
    const int n = s.n, k = s.k, kpad = s.kpad;
    g.n = n;
    g.nnz = s.nnz;
    g.k = k;
    g.kpad = kpad;
    g.first = s.first;
    g.W = s.dmax + 1;
    g.L = s.delta_max + 1;
    g.parity = s.parity;
    g.tol = s.tol;
    g.done0 = s.done;
    const int T = tile_cols(k);
    g.ntiles = T * (T + 1) / 2;
    g.nchunks = div_up(n, kPoolGramChunk);
    char* P = p->arena.base + s.off_p;
    Layout lp;
    g.rp = (const int*)(P + lp.add(sizeof(int) * (n + 1)));
    g.ci = (const int*)(P + lp.add(sizeof(int) * (size_t)std::max(s.nnz, 1)));
    g.pivots = (int*)(P + lp.add(sizeof(int) * kpad));
    g.dpk = (uint4*)(P + lp.add(sizeof(uint4) * (size_t)(kpad / 8) * n));
    g.delta = (int*)(P + lp.add(sizeof(int) * n));
    g.region = (int*)(P + lp.add(sizeof(int) * n));
    g.den64 = (double*)(P + lp.add(sizeof(double) * n));
    g.den32 = (float*)(P + lp.add(sizeof(float) * n));
    g.x64[0] = (double2*)(P + lp.add(sizeof(double2) * n));
    g.x64[1] = (double2*)(P + lp.add(sizeof(double2) * n));
    g.x32[0] = (float2*)(P + lp.add(sizeof(float2) * n));
    g.x32[1] = (float2*)(P + lp.add(sizeof(float2) * n));
    g.info = (int*)(P + lp.add(sizeof(int) * 8));
    if (s.off_s != kNone) {
        char* S = p->arena.base + s.off_s;
        Layout ls;
        g.ell = (int*)(S + ls.add(sizeof(int) * (size_t)n * kPoolEllW));
        g.dist = (int*)(S + ls.add(sizeof(int) * (size_t)k * n));
        g.m = (int*)(S + ls.add(sizeof(int) * n));
        g.gq = (int*)(S + ls.add(sizeof(int) * 3 * (size_t)n));
        g.colsum = (long long*)(S + ls.add(sizeof(long long) * k));
        g.mu = (double*)(S + ls.add(sizeof(double) * k));
        g.nu = (double*)(S + ls.add(sizeof(double) * n));
        g.stats = (double*)(S + ls.add(sizeof(double) * 4));
        g.M = (double*)(S + ls.add(sizeof(double) * (size_t)k * k));
        g.eig = (double*)(S + ls.add(sizeof(double) * (2 * (size_t)k + 2)));
        g.gpart = (double*)(S + ls.add(sizeof(double) * (size_t)g.nchunks * g.ntiles * 256));
    } else {
        g.ell = g.dist = g.m = g.gq = nullptr;
        g.colsum = nullptr;
        g.mu = g.nu = g.stats = g.M = g.eig = g.gpart = nullptr;
    }
    if (s.off_t != kNone) {
        char* T2 = p->arena.base + s.off_t;
        Layout lt;
        const size_t kw = (size_t)kpad * g.W;
        g.H = (int*)(T2 + lt.add(sizeof(int) * (size_t)k * g.W));
        g.w64 = (double*)(T2 + lt.add(sizeof(double) * kw));
        g.wt2 = (float2*)(T2 + lt.add(sizeof(float2) * kw));
        g.Hf = (float*)(T2 + lt.add(sizeof(float) * kw));
        g.invd = (float2*)(T2 + lt.add(sizeof(float2) * (size_t)g.W));
    } else {
        g.H = nullptr;
        g.w64 = nullptr;
        g.wt2 = nullptr;
        g.Hf = nullptr;
        g.invd = nullptr;
    }
    g.hist = pool_hist_mode(kpad, g.L, g.W);
}

size_t persist_bytes(int n, int nnz, int kpad) {
    Layout l;
    l.add(sizeof(int) * (n + 1));
    l.add(sizeof(int) * (size_t)std::max(nnz, 1));
    l.add(sizeof(int) * kpad);
    l.add(sizeof(uint4) * (size_t)(kpad / 8) * n);
    l.add(sizeof(int) * n);
    l.add(sizeof(int) * n);
    l.add(sizeof(double) * n);
    l.add(sizeof(float) * n);
    l.add(sizeof(double2) * n);
    l.add(sizeof(double2) * n);
    l.add(sizeof(float2) * n);
    l.add(sizeof(float2) * n);
    l.add(sizeof(int) * 8);
    return l.bytes;
}

size_t scratch_bytes(int n, int k) {
    const int T = tile_cols(k);
    Layout l;
    l.add(sizeof(int) * (size_t)n * kPoolEllW);
    l.add(sizeof(int) * (size_t)k * n);
    l.add(sizeof(int) * n);
    l.add(sizeof(int) * 3 * (size_t)n);
    l.add(sizeof(long long) * k);
    l.add(sizeof(double) * k);
    l.add(sizeof(double) * n);
    l.add(sizeof(double) * 4);
    l.add(sizeof(double) * (size_t)k * k);
    l.add(sizeof(double) * (2 * (size_t)k + 2));
    l.add(sizeof(double) * (size_t)div_up(n, kPoolGramChunk) * (T * (T + 1) / 2) * 256);
    return l.bytes;
}

size_t table_bytes(int k, int kpad, int W) {
    Layout l;
    l.add(sizeof(int) * (size_t)k * W);
    l.add(sizeof(double) * (size_t)kpad * W);
    l.add(sizeof(float2) * (size_t)kpad * W);
    l.add(sizeof(float) * (size_t)kpad * W);
    l.add(sizeof(float2) * (size_t)W);
    return l.bytes;
}

// What every kernel's memory accesses rely on: rows monotone from 0 to nnz
// and ids in [0, n).  Self-loops, duplicate and one-way arcs are found on the
// device during preparation (the graph then fails there).
ssm_status check_host_csr(int n, int nnz, const int* rp, const int* ci) {
    if (rp[0] != 0 || rp[n] != nnz) return fail(SSM_E_INVAL, "pool: row_ptr must run from 0 to nnz");
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(SSM_E_INVAL, "pool: row_ptr is not monotone");
    for (int e = 0; e < nnz; ++e)
        if ((unsigned)ci[e] >= (unsigned)n) return fail(SSM_E_INVAL, "pool: column index out of range");
    return SSM_OK;
}

Slot* get_slot(ssm_pool* p, int id) {
    if (id < 0 || id >= (int)p->slots.size() || p->slots[id].state == kFree) return nullptr;
    return &p->slots[id];
}

void release_scratch(ssm_pool* p, Slot& s) {
    p->arena.release(s.off_s, s.sz_s);
    s.off_s = kNone;
    s.sz_s = 0;
}

}  // namespace
}  // namespace ssm

using namespace ssm;

extern "C" {

ssm_status ssm_pool_create(int64_t capacity_bytes, ssm_pool** out) {
    if (!out) return fail(SSM_E_INVAL, "out is NULL");
    if (capacity_bytes < (int64_t)(1 << 20)) return fail(SSM_E_INVAL, "pool capacity below 1 MiB");
    ssm_pool* p = new ssm_pool();
    (void)hipGetDevice(&p->device);
    p->arena.cap = align_up((size_t)capacity_bytes);
    if (hipMalloc((void**)&p->arena.base, p->arena.cap) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(SSM_E_NOMEM, "pool: device allocation failed");
    }
    p->arena.free_[0] = p->arena.cap;
    const int T = kPoolMaxK / 16;
    std::vector<int2> ht;
    for (int b = 0; b < T; ++b)
        for (int a = 0; a <= b; ++a) ht.push_back(make_int2(a, b));
    hipError_t e = hipMalloc((void**)&p->tiles, sizeof(int2) * ht.size());
    if (e == hipSuccess) e = hipMemcpy(p->tiles, ht.data(), sizeof(int2) * ht.size(), hipMemcpyHostToDevice);
    for (auto& st : p->stage)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        ssm_pool_destroy(p);
        return hip_fail(e, "pool: create");
    }
    *out = p;
    return SSM_OK;
}

void ssm_pool_destroy(ssm_pool* p) {
    if (!p) return;
    (void)wait_all(p);
    for (auto& st : p->stage) {
        for (auto& kv : st.graphs) (void)hipGraphExecDestroy(kv.second);
        if (st.dev) (void)hipFree(st.dev);
        if (st.done) (void)hipEventDestroy(st.done);
    }
    if (p->capture) (void)hipStreamDestroy(p->capture);
    if (p->tiles) (void)hipFree(p->tiles);
    if (p->arena.base) (void)hipFree(p->arena.base);
    delete p;
}

ssm_status ssm_pool_usage(ssm_pool* p, int64_t* used, int64_t* capacity) {
    if (!p) return fail(SSM_E_INVAL, "pool is NULL");
    std::lock_guard<std::mutex> lk(p->mu);
    if (used) *used = (int64_t)p->arena.used;
    if (capacity) *capacity = (int64_t)p->arena.cap;
    return SSM_OK;
}

ssm_status ssm_pool_add(ssm_pool* p, int32_t n, int32_t nnz, const int32_t* row_ptr_host,
                        const int32_t* col_idx_host, int32_t k, int32_t first, int32_t sweeps, int32_t* slot_out,
                        hipStream_t stream) {
    if (!p || !row_ptr_host || (!col_idx_host && nnz > 0) || !slot_out) return fail(SSM_E_INVAL, "NULL argument");
    if (n < 1 || n > kPoolMaxN) return fail(SSM_E_RANGE, "pool graphs have 1 <= n <= 65536 nodes");
    if (nnz < 0) return fail(SSM_E_INVAL, "nnz < 0");
    if (k < 3 || k > n || k > kPoolMaxK) return fail(SSM_E_RANGE, "pool graphs need 3 <= k <= min(n, 256)");
    if (first < 0 || first >= n) return fail(SSM_E_INVAL, "first must lie in [0, n)");
    if (sweeps < 1) return fail(SSM_E_INVAL, "sweeps must be at least 1");
    ssm_status st = check_host_csr(n, nnz, row_ptr_host, col_idx_host);
    if (st != SSM_OK) return st;
    std::lock_guard<std::mutex> lk(p->mu);
    Slot s;
    s.n = n;
    s.nnz = nnz;
    s.k = k;
    s.kpad = div_up(k, 8) * 8;
    s.first = first;
    s.target = sweeps;
    s.sz_p = persist_bytes(n, nnz, s.kpad);
    s.sz_s = scratch_bytes(n, k);
    s.off_p = p->arena.alloc(s.sz_p);
    if (s.off_p != kNone) s.off_s = p->arena.alloc(s.sz_s);
    if (s.off_p == kNone || s.off_s == kNone) {
        p->arena.release(s.off_p, s.sz_p);
        return fail(SSM_E_NOMEM, "pool: capacity exhausted");
    }
    s.state = kAdded;
    bind(p, s);
    hipError_t e = hipMemcpyAsync((void*)s.g.rp, row_ptr_host, sizeof(int) * (n + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && nnz > 0)
        e = hipMemcpyAsync((void*)s.g.ci, col_idx_host, sizeof(int) * (size_t)nnz, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        p->arena.release(s.off_p, s.sz_p);
        p->arena.release(s.off_s, s.sz_s);
        return hip_fail(e, "pool: copy graph");
    }
    int id;
    if (!p->free_ids.empty()) {
        id = p->free_ids.back();
        p->free_ids.pop_back();
        p->slots[id] = s;
    } else {
        id = (int)p->slots.size();
        p->slots.push_back(s);
    }
    *slot_out = id;
    return SSM_OK;
}

ssm_status ssm_pool_prepare(ssm_pool* p, int32_t count, const int32_t* slots, int32_t warm, hipStream_t s) {
    if (!p || (count > 0 && !slots)) return fail(SSM_E_INVAL, "NULL argument");
    if (count < 0 || warm < 0) return fail(SSM_E_INVAL, "count and warm must be >= 0");
    std::lock_guard<std::mutex> lk(p->mu);
    std::vector<int> ids;
    for (int q = 0; q < count; ++q) {
        Slot* sl = get_slot(p, slots[q]);
        if (!sl || sl->state != kAdded) return fail(SSM_E_INVAL, "pool: prepare needs slots that are added, not yet prepared");
        for (int r : ids)
            if (r == slots[q]) return fail(SSM_E_INVAL, "pool: a slot is listed twice");
        ids.push_back(slots[q]);
    }
    if (ids.empty()) return SSM_OK;
    // per-call device buffers: descriptors, BFS items, Gram items, BFS
    // overflow queues, info copy
    int nmax = 0, kmax = 0, kpmax = 0;
    long long nbfs = 0, ngram = 0;
    for (int id : ids) {
        const Slot& sl = p->slots[id];
        nmax = std::max(nmax, sl.n);
        kmax = std::max(kmax, sl.k);
        kpmax = std::max(kpmax, tile_cols(sl.k) * 16);
        nbfs += sl.k;
        const int T = tile_cols(sl.k);
        ngram += (long long)div_up(sl.n, kPoolGramChunk) * div_up(T * (T + 1) / 2, 32);
    }
    const int nq = (int)ids.size();
    const int bfs_blocks = pool_bfs_blocks((int)nbfs);
    const long long gq_stride = 3LL * nmax;
    Layout lw;
    const size_t o_g = lw.add(sizeof(PoolGraph) * nq), o_bi = lw.add(sizeof(int2) * nbfs),
                 o_gi = lw.add(sizeof(int4) * ngram), o_q = lw.add(sizeof(int) * gq_stride * bfs_blocks),
                 o_info = lw.add(sizeof(int) * 8 * nq);
    long long nitems = 0;  // 256-node items of the FP64 stages
    for (int id : ids) nitems += div_up(p->slots[id].n, 256);
    const size_t o_it = lw.add(sizeof(int2) * nitems);
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, lw.bytes);
    if (st != SSM_OK) return st;
    PoolGraph* dg = (PoolGraph*)(ws + o_g);
    int2* dbi = (int2*)(ws + o_bi);
    int4* dgi = (int4*)(ws + o_gi);
    int* dq = (int*)(ws + o_q);
    int* dinfo = (int*)(ws + o_info);
    int2* dit = (int2*)(ws + o_it);
    std::vector<PoolGraph> hg(nq);
    std::vector<int2> hbi, hit;
    std::vector<int4> hgi;
    for (int q = 0; q < nq; ++q) {
        Slot& sl = p->slots[ids[q]];
        bind(p, sl);
        hg[q] = sl.g;
        for (int t = 0; t < sl.k; ++t) hbi.push_back(make_int2(q, t));
        for (int i0 = 0; i0 < sl.n; i0 += 256) hit.push_back(make_int2(q, i0));
    }
    hipError_t e = hipMemcpyAsync(dg, hg.data(), sizeof(PoolGraph) * nq, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dbi, hbi.data(), sizeof(int2) * nbfs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dit, hit.data(), sizeof(int2) * nitems, hipMemcpyHostToDevice, s);
    // stage 1: CSR checks, selection and BFS
    if (e == hipSuccess) e = pool_prep_init(dg, nq, nmax, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pool_validate, dim3((int)nitems), dim3(256), 0, s, dg, dit);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = pool_select(dg, nq, nmax, s);
    if (e == hipSuccess) e = pool_bfs(dg, dbi, (int)nbfs, dq, gq_stride, bfs_blocks, s);
    std::vector<int> hinfo(8 * (size_t)nq);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pool_gather_info, dim3(div_up(8 * nq, 256)), dim3(256), 0, s, dg, nq, dinfo);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hinfo.data(), dinfo, sizeof(int) * 8 * nq, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // stage 2: tables for the connected graphs, then regions, terms,
    // PivotMDS and the FP64 warm-up sweeps
    std::vector<int> ok;  // positions in ids
    if (e == hipSuccess) {
        for (int q = 0; q < nq; ++q) {
            Slot& sl = p->slots[ids[q]];
            if (hinfo[8 * q + 5] != 0) {
                sl.state = kFailed;
                sl.fail = SSM_E_INVAL;  // not a simple undirected graph
                continue;
            }
            if (hinfo[8 * q] != 0) {
                sl.state = kFailed;
                sl.fail = SSM_E_DISCONNECTED;
                continue;
            }
            sl.dmax = hinfo[8 * q + 1];
            sl.sz_t = table_bytes(sl.k, sl.kpad, sl.dmax + 1);
            sl.off_t = p->arena.alloc(sl.sz_t);
            if (sl.off_t == kNone) {
                sl.state = kFailed;
                sl.fail = SSM_E_NOMEM;
                continue;
            }
            bind(p, sl);
            hg[q] = sl.g;
            ok.push_back(q);
        }
    }
    if (e == hipSuccess && !ok.empty()) {
        // compact the descriptors of the graphs that go on
        std::vector<PoolGraph> h2;
        std::vector<int4> hgi2;
        std::vector<int2> hit2;
        int kmx = 0, kpmx = 0, nmx = 0;
        for (size_t r = 0; r < ok.size(); ++r) {
            const Slot& sl = p->slots[ids[ok[r]]];
            h2.push_back(hg[ok[r]]);
            kmx = std::max(kmx, sl.k);
            kpmx = std::max(kpmx, tile_cols(sl.k) * 16);
            nmx = std::max(nmx, sl.n);
            const int T = tile_cols(sl.k), ng = div_up(T * (T + 1) / 2, 32);
            for (int c = 0; c < div_up(sl.n, kPoolGramChunk); ++c)
                for (int grp = 0; grp < ng; ++grp) hgi2.push_back(make_int4((int)r, c, grp, 0));
            for (int i0 = 0; i0 < sl.n; i0 += 256) hit2.push_back(make_int2((int)r, i0));
        }
        const int nok = (int)ok.size();
        e = hipMemcpyAsync(dg, h2.data(), sizeof(PoolGraph) * nok, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(dgi, hgi2.data(), sizeof(int4) * hgi2.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(dit, hit2.data(), sizeof(int2) * hit2.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            const size_t lds = sizeof(int) * 2 * (size_t)kmx + sizeof(unsigned) * (size_t)div_up(nmx, 32) +
                               sizeof(unsigned short) * (size_t)nmx;
            if (lds > 64 * 1024)
                (void)hipFuncSetAttribute((const void*)k_pool_regions, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds);
            hipLaunchKernelGGL(k_pool_regions, dim3(nok), dim3(1024), lds, s, dg);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = pool_pivotmds(dg, nok, dgi, (int)hgi2.size(), p->tiles, kpmx, kmx, s);
        int src = 0;
        for (int w = 0; w < warm && e == hipSuccess; ++w, src ^= 1) {
            hipLaunchKernelGGL(k_pool_sweep64, dim3((int)hit2.size()), dim3(256), 0, s, dg, dit, src);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_pool_round, dim3((int)hit2.size()), dim3(256), 0, s, dg, dit, src);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_pool_gather_info, dim3(div_up(8 * nok, 256)), dim3(256), 0, s, dg, nok, dinfo);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(hinfo.data(), dinfo, sizeof(int) * 8 * nok, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) {
            for (int r = 0; r < nok; ++r) {
                Slot& sl = p->slots[ids[ok[r]]];
                sl.delta_max = hinfo[8 * r + 2];
                if (hinfo[8 * r + 3] != 0) {
                    sl.state = kFailed;
                    sl.fail = SSM_E_INVAL;  // zero total edge length
                    continue;
                }
                sl.state = kReady;
                sl.done = warm;
                sl.parity = 0;
                sl.x64cur = warm & 1;
            }
        }
    }
    (void)hipStreamSynchronize(s);  // idle before scratch and per-call buffers are reused
    sfree(ws);
    for (int id : ids) {
        Slot& sl = p->slots[id];
        release_scratch(p, sl);
        if (sl.state == kAdded) {  // stopped by an error before it was decided
            sl.state = kFailed;
            sl.fail = SSM_E_DEVICE;
        }
        bind(p, sl);
    }
    if (e != hipSuccess) return hip_fail(e, "pool: prepare");
    return SSM_OK;
}

ssm_status ssm_pool_sweep(ssm_pool* p, int32_t count, const int32_t* slots, int32_t iters, hipStream_t s) {
    if (!p || (count > 0 && !slots)) return fail(SSM_E_INVAL, "NULL argument");
    if (count < 0 || iters < 0) return fail(SSM_E_INVAL, "count and iters must be >= 0");
    std::lock_guard<std::mutex> lk(p->mu);
    for (int q = 0; q < count; ++q) {
        Slot* sl = get_slot(p, slots[q]);
        if (!sl || sl->state != kReady) return fail(SSM_E_INVAL, "pool: sweep needs prepared slots");
        for (int r = 0; r < q; ++r)
            if (slots[r] == slots[q]) return fail(SSM_E_INVAL, "pool: a slot is listed twice");
    }
    if (count == 0 || iters == 0) return SSM_OK;
    Stage& stg = p->stage[p->flip];
    ssm_status st = wait_stage(stg);
    if (st != SSM_OK) return st;
    stg.hg.clear();
    stg.hc.clear();
    int most = 0;
    size_t lds = 0;
    bool any_tol = false;
    std::vector<int> first;  // first chunk of each listed graph (for the stop test)
    for (int q = 0; q < count; ++q) {
        Slot& sl = p->slots[slots[q]];
        PoolGraph g = sl.g;
        g.iters = std::max(0, std::min(iters, sl.target - sl.done));
        g.parity = sl.parity;
        g.tol = sl.tol;
        g.done0 = sl.done;
        any_tol = any_tol || (sl.tol > 0.0 && g.iters > 0);
        most = std::max(most, g.iters);
        stg.hg.push_back(g);
        first.push_back((int)stg.hc.size());
        for (int i0 = 0; i0 < sl.n; i0 += kPoolSweepBlock) stg.hc.push_back(make_int2(q, i0));
        lds = std::max(lds, sizeof(float2) * (size_t)sl.kpad +
                                (g.hist ? sizeof(float2) * (size_t)g.W + sizeof(float) * (size_t)sl.kpad * g.L : 0));
    }
    if (most == 0) return SSM_OK;
    first.push_back((int)stg.hc.size());
    const int nch = (int)stg.hc.size();
    // Launch grids rounded up to a multiple of an eighth of the next power of
    // two (at most a quarter more blocks, which return at once), so that one
    // captured graph serves every quantum whose counts round alike (variant
    // pool_graph -1: direct launches over the exact grids)
    const bool use_graph = !p->no_graphs && variant("pool_graph") != -1;
    auto bucket = [&](int v) {
        if (!use_graph) return v;
        int b = 16;
        while (b < v) b <<= 1;
        const int q = std::max(4, b / 8);  // steps of an eighth of the octave's top
        return std::max(16, div_up(v, q) * q);
    };
    const int nchB = bucket(nch), countB = bucket(count);
    const size_t ldsB = use_graph ? (size_t)div_up((long long)lds, 4096) * 4096 : lds;
    // stage layout: header (chunk and graph counts), graphs, chunks, first
    // chunk per graph, moment partials; offsets from the rounded counts
    const size_t o_g = 256;
    const size_t o_c = o_g + align_up(sizeof(PoolGraph) * countB);
    const size_t o_first = o_c + align_up(sizeof(int2) * nchB);
    const size_t o_part = o_first + align_up(sizeof(int) * (countB + 1));
    const size_t need = any_tol ? o_part + sizeof(double) * kMoments * nchB : o_first;
    if (need > stg.cap) {
        const size_t want = std::max(need, stg.cap * 2);
        for (auto& kv : stg.graphs) (void)hipGraphExecDestroy(kv.second);  // they point into the old buffer
        stg.graphs.clear();
        if (stg.dev) (void)hipFree(stg.dev);
        stg.dev = nullptr;
        stg.cap = 0;
        if (hipMalloc((void**)&stg.dev, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SSM_E_NOMEM, "pool: sweep staging buffer");
        }
        stg.cap = want;
    }
    int* dh = (int*)stg.dev;
    PoolGraph* dg = (PoolGraph*)(stg.dev + o_g);
    int2* dc = (int2*)(stg.dev + o_c);
    int* dfirst = any_tol ? (int*)(stg.dev + o_first) : nullptr;
    double* dpart = any_tol ? (double*)(stg.dev + o_part) : nullptr;
    const int hdr[4] = {nch, count, 0, 0};
    hipError_t e = hipMemcpyAsync(dh, hdr, sizeof hdr, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dg, stg.hg.data(), sizeof(PoolGraph) * stg.hg.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dc, stg.hc.data(), sizeof(int2) * stg.hc.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && any_tol)
        e = hipMemcpyAsync(dfirst, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, s);
    if (ldsB > 64 * 1024) {
        (void)hipFuncSetAttribute((const void*)k_pool_sweep32<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ldsB);
        (void)hipFuncSetAttribute((const void*)k_pool_sweep32<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ldsB);
    }
    // persistent grid: the blocks of k_pool_sweep32 resident at once
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_pool_sweep32<true>, kPoolSweepBlock,
                                                     ldsB) != hipSuccess)
        occ = 1;
    const int pgrid = std::max(1, occ) * num_cus();
    auto launch_sweep = [&](hipStream_t q, int it, bool persist, int grid_c, int grid_g) {
        if (persist)
            hipLaunchKernelGGL(k_pool_sweep32<true>, dim3(pgrid), dim3(kPoolSweepBlock), ldsB, q, dg, dc, dh, it);
        else
            hipLaunchKernelGGL(k_pool_sweep32<false>, dim3(grid_c), dim3(kPoolSweepBlock), ldsB, q, dg, dc, dh, it);
        if (any_tol) {
            hipLaunchKernelGGL(k_pool_moments, dim3(grid_c), dim3(256), 0, q, dg, dc, dh, it, dpart);
            hipLaunchKernelGGL(k_pool_decide, dim3(div_up((long long)grid_g * kWave, 256)), dim3(256), 0, q, dg, dh,
                               dfirst, dpart, it);
        }
    };
    // Schedule: a block per chunk or a persistent grid (variant pool_persist
    // 1 | -1 forces one).  Both give the same layouts bit for bit; the first
    // call of a shape class with at least 4 sweeps times its sweeps 0-3
    // alternately with each schedule and keeps the persistent grid for the
    // class only if it was at least 5 % faster (the timings share the device
    // with preparation work on other streams; on the serving stream a block
    // per chunk measured faster: 4210-4228 against 3944-3960 layouts/s).
    int from = 0;  // sweeps already launched
    const int pv = variant("pool_persist");
    bool persist = pv == 1;
    if (pv == 0 && e == hipSuccess) {
        const ScheduleKey sk{bucket(nch), bucket(count), (int)ldsB};
        auto known = p->schedule.find(sk);
        if (known != p->schedule.end()) {
            persist = known->second != 0;
        } else if (most >= 4) {
            hipEvent_t ev[5] = {};
            hipError_t c = hipSuccess;
            for (int q = 0; q < 5 && c == hipSuccess; ++q) c = hipEventCreate(&ev[q]);
            if (c == hipSuccess) c = hipEventRecord(ev[0], s);
            for (int it = 0; it < 4 && c == hipSuccess; ++it) {
                launch_sweep(s, it, (it & 1) != 0, nch, count);
                c = hipGetLastError();
                if (c == hipSuccess) c = hipEventRecord(ev[it + 1], s);
            }
            if (c == hipSuccess) c = hipEventSynchronize(ev[4]);
            float ms[4] = {0.f, 0.f, 0.f, 0.f};
            for (int it = 0; it < 4 && c == hipSuccess; ++it) c = hipEventElapsedTime(&ms[it], ev[it], ev[it + 1]);
            for (auto& v : ev)
                if (v) (void)hipEventDestroy(v);
            if (c != hipSuccess) {
                e = c;
            } else {
                persist = ms[1] + ms[3] < 0.95f * (ms[0] + ms[2]);
                p->schedule[sk] = persist ? 1 : 0;
                from = 4;
            }
        }
    }
    auto launch_quantum = [&](hipStream_t q, int grid_c, int grid_g) {
        for (int it = from; it < most; ++it) launch_sweep(q, it, persist, grid_c, grid_g);
    };
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess && use_graph && from == 0) {
        const QuantumKey key{nchB, countB, most, (int)ldsB, any_tol ? 1 : 0, persist ? 1 : 0};
        auto it = stg.graphs.find(key);
        if (it != stg.graphs.end()) {
            exec = it->second;
        } else {
            // capture on the pool's own stream (the caller's may be the null
            // stream, which cannot be captured); nothing runs there
            hipError_t c = p->capture ? hipSuccess : hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
            hipGraph_t graph = nullptr;
            if (c == hipSuccess) c = hipStreamBeginCapture(p->capture, hipStreamCaptureModeRelaxed);
            if (c == hipSuccess) {
                launch_quantum(p->capture, nchB, countB);
                c = hipStreamEndCapture(p->capture, &graph);
            }
            if (c == hipSuccess) c = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (c == hipSuccess) {
                stg.graphs[key] = exec;
            } else {  // no graphs from now on; this quantum launches directly
                (void)hipGetLastError();
                exec = nullptr;
                p->no_graphs = true;
            }
        }
    }
    if (e == hipSuccess) {
        if (exec)
            e = hipGraphLaunch(exec, s);
        else {
            launch_quantum(s, nch, count);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipEventRecord(stg.done, s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        return hip_fail(e, "pool: sweep");
    }
    stg.pending = true;
    p->flip ^= 1;
    for (int q = 0; q < count; ++q) {
        Slot& sl = p->slots[slots[q]];
        const int d = stg.hg[q].iters;
        sl.done += d;
        sl.parity = (sl.parity + d) & 1;
        sl.g.parity = sl.parity;
    }
    return SSM_OK;
}

ssm_status ssm_pool_set_tol(ssm_pool* p, int32_t slot, double tol) {
    if (!p) return fail(SSM_E_INVAL, "pool is NULL");
    if (!(tol >= 0.0)) return fail(SSM_E_INVAL, "tol must be >= 0");
    std::lock_guard<std::mutex> lk(p->mu);
    Slot* sl = get_slot(p, slot);
    if (!sl || (sl->state != kAdded && sl->state != kReady)) return fail(SSM_E_INVAL, "pool: no such slot");
    sl->tol = tol;
    sl->g.tol = tol;
    return SSM_OK;
}

ssm_status ssm_pool_stopped(ssm_pool* p, int32_t count, const int32_t* slots, int32_t* sweeps_host,
                            hipStream_t s) {
    if (!p || (count > 0 && (!slots || !sweeps_host))) return fail(SSM_E_INVAL, "NULL argument");
    if (count < 0) return fail(SSM_E_INVAL, "count must be >= 0");
    std::lock_guard<std::mutex> lk(p->mu);
    std::vector<PoolGraph> hg;
    for (int q = 0; q < count; ++q) {
        Slot* sl = get_slot(p, slots[q]);
        if (!sl || sl->state != kReady) return fail(SSM_E_INVAL, "pool: stopped needs prepared slots");
        hg.push_back(sl->g);
    }
    if (count == 0) return SSM_OK;
    ssm_status st = wait_all(p);  // the slots' last sweeps may run on another stream
    if (st != SSM_OK) return st;
    char* ws = nullptr;
    const size_t o_info = align_up(sizeof(PoolGraph) * count);
    st = salloc((void**)&ws, o_info + sizeof(int) * 8 * (size_t)count);
    if (st != SSM_OK) return st;
    std::vector<int> hinfo(8 * (size_t)count);
    hipError_t e = hipMemcpyAsync(ws, hg.data(), sizeof(PoolGraph) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pool_gather_info, dim3(div_up(8 * count, 256)), dim3(256), 0, s, (const PoolGraph*)ws,
                           count, (int*)(ws + o_info));
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(hinfo.data(), ws + o_info, sizeof(int) * 8 * (size_t)count, hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "pool: stopped");
    if (e2 != hipSuccess) return hip_fail(e2, "pool: stopped");
    for (int q = 0; q < count; ++q) {
        Slot& sl = p->slots[slots[q]];
        if (hinfo[8 * (size_t)q + 6]) {
            sweeps_host[q] = hinfo[8 * (size_t)q + 7];
            sl.target = sl.done;  // no further sweeps
        } else {
            sweeps_host[q] = -1;
        }
    }
    return SSM_OK;
}

ssm_status ssm_pool_stress(ssm_pool* p, int32_t count, const int32_t* slots, double* out_host, hipStream_t s) {
    if (!p || (count > 0 && (!slots || !out_host))) return fail(SSM_E_INVAL, "NULL argument");
    if (count < 0) return fail(SSM_E_INVAL, "count must be >= 0");
    std::lock_guard<std::mutex> lk(p->mu);
    std::vector<PoolGraph> hg;
    std::vector<int2> hc;
    std::vector<int> first;
    for (int q = 0; q < count; ++q) {
        Slot* sl = get_slot(p, slots[q]);
        if (!sl || sl->state != kReady) return fail(SSM_E_INVAL, "pool: stress needs prepared slots");
        hg.push_back(sl->g);
        first.push_back((int)hc.size());
        for (int i0 = 0; i0 < sl->n; i0 += kWave) hc.push_back(make_int2(q, i0));
    }
    first.push_back((int)hc.size());
    if (count == 0) return SSM_OK;
    ssm_status st0 = wait_all(p);  // the slots' last sweeps may run on another stream
    if (st0 != SSM_OK) return st0;
    Layout l;
    const size_t o_g = l.add(sizeof(PoolGraph) * count), o_c = l.add(sizeof(int2) * hc.size()),
                 o_f = l.add(sizeof(int) * first.size()), o_p = l.add(sizeof(double) * hc.size()),
                 o_o = l.add(sizeof(double) * count);
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, l.bytes);
    if (st != SSM_OK) return st;
    hipError_t e = hipMemcpyAsync(ws + o_g, hg.data(), sizeof(PoolGraph) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + o_c, hc.data(), sizeof(int2) * hc.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + o_f, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        const int nch = (int)hc.size();
        hipLaunchKernelGGL(k_pool_stress, dim3(div_up(nch, 4)), dim3(256), 0, s, (const PoolGraph*)(ws + o_g),
                           (const int2*)(ws + o_c), nch, (double*)(ws + o_p));
        hipLaunchKernelGGL(k_pool_stress_sum, dim3(div_up(count, 64)), dim3(64), 0, s, count,
                           (const int*)(ws + o_f), (const double*)(ws + o_p), (double*)(ws + o_o));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, ws + o_o, sizeof(double) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "pool: stress");
    return SSM_OK;
}

ssm_status ssm_pool_layout(ssm_pool* p, int32_t slot, float* x_out, hipStream_t s) {
    if (!p || !x_out) return fail(SSM_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    Slot* sl = get_slot(p, slot);
    if (!sl || sl->state != kReady) return fail(SSM_E_INVAL, "pool: layout needs a prepared slot");
    ssm_status st = wait_all(p);  // the slot's last sweep may run on another stream
    if (st != SSM_OK) return st;
    SSM_HIP(hipMemcpyAsync(x_out, sl->g.x32[sl->parity], sizeof(float2) * sl->n, hipMemcpyDeviceToDevice, s));
    return SSM_OK;
}

ssm_status ssm_pool_export(ssm_pool* p, int32_t slot, int32_t what, void* host_out, hipStream_t s) {
    if (!p || !host_out) return fail(SSM_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    Slot* sl = get_slot(p, slot);
    if (!sl || sl->state != kReady) return fail(SSM_E_INVAL, "pool: export needs a prepared slot");
    ssm_status st = wait_all(p);
    if (st != SSM_OK) return st;
    const PoolGraph& g = sl->g;
    const size_t n = sl->n, k = sl->k, W = sl->dmax + 1, L = sl->delta_max + 1;
    const void* src = nullptr;
    size_t bytes = 0;
    std::vector<uint4> words;
    switch (what) {
        case SSM_POOL_PIVOTS: src = g.pivots; bytes = sizeof(int) * k; break;
        case SSM_POOL_DELTA: src = g.delta; bytes = sizeof(int) * n; break;
        case SSM_POOL_REGION: src = g.region; bytes = sizeof(int) * n; break;
        case SSM_POOL_H: src = g.H; bytes = sizeof(int) * k * L; break;
        case SSM_POOL_WTAB64: src = g.w64; bytes = sizeof(double) * k * W; break;
        case SSM_POOL_DEN64: src = g.den64; bytes = sizeof(double) * n; break;
        case SSM_POOL_X32: src = g.x32[sl->parity]; bytes = sizeof(float2) * n; break;
        case SSM_POOL_X64: src = g.x64[sl->x64cur]; bytes = sizeof(double2) * n; break;
        case SSM_POOL_DIST: {
            words.resize((size_t)(sl->kpad / 8) * n);
            SSM_HIP(hipMemcpyAsync(words.data(), g.dpk, sizeof(uint4) * words.size(), hipMemcpyDeviceToHost, s));
            SSM_HIP(hipStreamSynchronize(s));
            int32_t* out = (int32_t*)host_out;
            for (size_t t = 0; t < k; ++t)
                for (size_t i = 0; i < n; ++i) {
                    const uint16_t* e = (const uint16_t*)&words[(t / 8) * n + i];
                    out[t * n + i] = e[t % 8];
                }
            return SSM_OK;
        }
        default: return fail(SSM_E_INVAL, "pool: unknown export");
    }
    SSM_HIP(hipMemcpyAsync(host_out, src, bytes, hipMemcpyDeviceToHost, s));
    SSM_HIP(hipStreamSynchronize(s));
    return SSM_OK;
}

ssm_status ssm_pool_info(ssm_pool* p, int32_t slot, int32_t* info_host) {
    if (!p || !info_host) return fail(SSM_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    Slot* sl = get_slot(p, slot);
    if (!sl) return fail(SSM_E_INVAL, "pool: no such slot");
    const int32_t v[8] = {sl->state, sl->fail, sl->n, sl->k, sl->done, sl->target, sl->dmax, sl->delta_max};
    for (int q = 0; q < 8; ++q) info_host[q] = v[q];
    return SSM_OK;
}

ssm_status ssm_pool_remove(ssm_pool* p, int32_t slot) {
    if (!p) return fail(SSM_E_INVAL, "pool is NULL");
    std::lock_guard<std::mutex> lk(p->mu);
    Slot* sl = get_slot(p, slot);
    if (!sl) return fail(SSM_E_INVAL, "pool: no such slot");
    ssm_status st = wait_all(p);  // no queued sweep may still read the slot
    if (st != SSM_OK) return st;
    p->arena.release(sl->off_p, sl->sz_p);
    p->arena.release(sl->off_s, sl->sz_s);
    p->arena.release(sl->off_t, sl->sz_t);
    *sl = Slot();
    p->free_ids.push_back(slot);
    return SSM_OK;
}

}  // extern "C"
