// Breadth-first searches from the pivots, max/min pivot sampling and the
// nearest-pivot regions R(p) (paper Section 3 and Section 4.1).
#include <hip/hip_cooperative_groups.h>
#include <limits.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "ssm_internal.h"
#include "wave.h"

namespace cg = cooperative_groups;

namespace ssm {

constexpr int kBfsBlock = 1024;
constexpr int kSelBlock = 512;
constexpr int kInf = INT_MAX;


// Lanes per frontier node: the power of two nearest the mean degree, in [2, 64].
static int virtual_warp(const ssm_csr* g) {
    int forced = variant("bfs_lanes");
    if (forced == 2 || forced == 4 || forced == 8 || forced == 16 || forced == 32 || forced == 64) return forced;
    double avg = g->n > 0 ? (double)g->nnz / g->n : 1.0;
    int vw = 2;
    while (vw < 64 && vw < avg) vw <<= 1;
    return vw;
}

// Fills p[0..count) with v.
__global__ void k_fill_int(int* p, int v, long long count) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------ validation

// Rows: row_ptr monotone from 0 to nnz.
__global__ void k_validate_rows(int n, int nnz, const int* __restrict__ rp, int* bad) {
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const int a = rp[u], b = rp[u + 1];
        if (a < 0 || b < a || b > nnz || (u == 0 && a != 0) || (u == n - 1 && b != nnz)) atomicOr(bad, 1);
    }
}

// Every arc (u, v), one thread each (launched once the rows are known to be
// valid): v in range, v != u, and the reverse arc (v, u) present exactly once
// in row v and (u, v) exactly once in row u (this also rejects duplicate
// arcs).  The rows are scanned linearly, so they need not be sorted; the
// work is sum over arcs of both rows' lengths, spread over all threads (a
// thread per node would serialize a hub's squared degree in one thread).
__global__ void k_validate_arcs(int n, int nnz, const int* __restrict__ rp, const int* __restrict__ ci, int* bad) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz;
         e += (long long)gridDim.x * blockDim.x) {
        int lo = 0, hi = n - 1;  // the row holding arc e: the last u with rp[u] <= e
        while (lo < hi) {
            const int mid = (int)(((long long)lo + hi + 1) >> 1);
            if (rp[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int u = lo, a = rp[u], b = rp[u + 1];
        const int v = ci[e];
        if (v < 0 || v >= n || v == u) {
            atomicOr(bad, 2);
            continue;
        }
        const int c0 = rp[v], c1 = rp[v + 1];
        int hits = 0;
        for (int f = c0; f < c1; ++f) hits += (ci[f] == u);
        int same = 0;
        for (int f = a; f < b; ++f) same += (ci[f] == v);
        if (hits != 1 || same != 1) atomicOr(bad, 4);
    }
}

// ------------------------------------------------- one BFS per workgroup

// Frontier queue of one workgroup: the first kQcap entries live in LDS, the
// rest in a global overflow area of n entries.  An entry is the row bounds
// (row_ptr[v], row_ptr[v+1]) of a frontier node, loaded when the node is
// pushed, so that the next level starts with its neighbour loads.
constexpr int kQcap = 3072;
constexpr int kBfsU = 4;

// Agent-scope relaxed loads compile to cache-bypassing (sc1) loads.  They
// are coherent with every block's atomics and agent-scope stores, and on
// MI355X a chain of them measures about 90 ns per dependent load against
// about 350 ns for plain loads that miss L2, so the BFS kernels take their
// latency-bound loads (row bounds, neighbour ids, visited checks) this way.
__device__ __forceinline__ int load_agent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int wg_load(const int* p) {  // coherent with this workgroup's atomics (and all others')
    return load_agent(p);
}

__device__ __forceinline__ int2 queue_get(const int2* lds, const int2* glob, int idx) {
    if (idx < kQcap) return lds[idx];
    const int* g = (const int*)(glob + (idx - kQcap));
    return make_int2(wg_load(g), wg_load(g + 1));
}

// Loads of the read-only CSR arrays: agent-scope (AG) or plain, cached
// loads.
template <bool AG>
__device__ __forceinline__ int csr_load(const int* p) {
    if (AG) return load_agent(p);
    return *p;
}

// Row bounds of the frontier entry `q`: stored directly (ROWQ) or looked up
// from the stored node id (entry.x).
template <bool ROWQ, bool AG = true>
__device__ __forceinline__ int2 entry_row(int2 q, const int* __restrict__ rp, int n) {
    if (ROWQ) return q;
    return (unsigned)q.x < (unsigned)n ? make_int2(csr_load<AG>(&rp[q.x]), csr_load<AG>(&rp[q.x + 1]))
                                       : make_int2(0, 0);
}

template <bool ROWQ, bool AG = true>
__device__ __forceinline__ int2 make_entry(int v, const int* __restrict__ rp) {
    if (ROWQ) return make_int2(csr_load<AG>(&rp[v]), csr_load<AG>(&rp[v + 1]));
    return make_int2(v, 0);
}

__device__ __forceinline__ void queue_put(int2* lds, int2* glob, int idx, int2 v) {
    if (idx < kQcap)
        lds[idx] = v;
    else
        glob[idx - kQcap] = v;
}

// Block b runs a level-synchronous BFS from pivots[b] and writes
// dist[b][*] (pre-set to -1).  Frontier nodes are spread over groups of VW
// lanes; a node is claimed by compare-and-swap on its distance (workgroup
// scope: the row belongs to this block) and appended to the next frontier
// with one LDS atomic per wave.  LD picks the loads: 0 = agent-scope loads
// throughout; 1 = plain (cached) loads of the read-only CSR arrays; 2 = also
// the visited check as a plain load (a stale "unvisited" costs only a failed
// swap).  reached[b] = nodes found; *ecc_max = largest eccentricity seen.
template <int VW, bool ROWQ, int LD>
__global__ __launch_bounds__(kBfsBlock) void k_bfs_wg(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const int* __restrict__ pivots, int* dist,
                                                      int2* queues, int* reached, int* ecc_max) {
    constexpr bool AG = LD == 0;
    const int b = blockIdx.x;
    int* D = dist + (size_t)b * n;
    int2* ga = queues + (size_t)b * 2 * n;
    int2* gb = ga + n;
    __shared__ int2 sqa[kQcap], sqb[kQcap];
    __shared__ int s_tail, s_len;
    const int src = pivots[b];
    if (threadIdx.x == 0) {
        D[src] = 0;
        sqa[0] = make_entry<ROWQ, AG>(src, rp);
        s_len = 1;
        s_tail = 0;
    }
    __syncthreads();
    const int sub = threadIdx.x % VW, grp = threadIdx.x / VW, ngrp = blockDim.x / VW;
    int2* lcur = sqa;
    int2* lnxt = sqb;
    int2* gcur = ga;
    int2* gnxt = gb;
    int level = 0, total = 1;
    for (;;) {
        const int len = min(s_len, n);
        if (len == 0) break;
        // kBfsU frontier entries per lane group and pass, their loads in flight
        // together (a level is a few passes of dependent memory round trips)
        for (int base = 0; base < len; base += ngrp * kBfsU) {
            int2 row[kBfsU];
            int span = 0;
#pragma unroll
            for (int q = 0; q < kBfsU; ++q) {
                const int qi = base + q * ngrp + grp;
                row[q] = qi < len ? entry_row<ROWQ, AG>(queue_get(lcur, gcur, qi), rp, n) : make_int2(0, 0);
                span = max(span, row[q].y - row[q].x);
            }
            for (int j = sub; j < span; j += VW) {
                int v[kBfsU], seen[kBfsU];
#pragma unroll
                for (int q = 0; q < kBfsU; ++q) v[q] = row[q].x + j < row[q].y ? csr_load<AG>(&ci[row[q].x + j]) : -1;
#pragma unroll
                for (int q = 0; q < kBfsU; ++q)
                    seen[q] = (unsigned)v[q] < (unsigned)n ? (LD == 2 ? *(const int*)&D[v[q]] : wg_load(&D[v[q]])) : 0;
                bool claim[kBfsU];
#pragma unroll
                for (int q = 0; q < kBfsU; ++q) {
                    claim[q] = false;
                    if ((unsigned)v[q] < (unsigned)n && seen[q] < 0) {
                        int expected = -1;
                        claim[q] = __hip_atomic_compare_exchange_strong(&D[v[q]], &expected, level + 1,
                                                                        __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                int2 vrow[kBfsU];
#pragma unroll
                for (int q = 0; q < kBfsU; ++q)
                    if (claim[q]) vrow[q] = make_entry<ROWQ, AG>(v[q], rp);
#pragma unroll
                for (int q = 0; q < kBfsU; ++q) {
                    const int slot = wave_append(claim[q], &s_tail);
                    if (claim[q]) queue_put(lnxt, gnxt, slot, vrow[q]);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_len = s_tail;
            s_tail = 0;
        }
        int2* t0 = lcur;
        lcur = lnxt;
        lnxt = t0;
        int2* t1 = gcur;
        gcur = gnxt;
        gnxt = t1;
        ++level;
        __syncthreads();
        total += s_len;
    }
    if (threadIdx.x == 0) {
        reached[b] = total;
        atomicMax(ecc_max, level - 1);
    }
}

// Ids of the nodes with degree > kHeavyDegree in ascending order: blocks
// count their range, a single thread scans the counts, blocks write their ids
// at their offset (ballot compaction keeps the id order inside a block).
constexpr int kHeavySpan = 4096;  // nodes per block

__global__ __launch_bounds__(256) void k_heavy_count(int n, const int* __restrict__ rp, int* __restrict__ counts) {
    const int i0 = blockIdx.x * kHeavySpan;
    int c = 0;
    for (int i = i0 + threadIdx.x; i < min(n, i0 + kHeavySpan); i += blockDim.x) c += rp[i + 1] - rp[i] > kHeavyDegree;
    __shared__ int red[256 / kWave];
    c = block_sum(c, red);
    if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

__global__ void k_heavy_scan(int nb, int* __restrict__ counts, int* __restrict__ total) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int acc = 0;
        for (int b = 0; b < nb; ++b) {
            int c = counts[b];
            counts[b] = acc;
            acc += c;
        }
        total[0] = acc;
    }
}

__global__ __launch_bounds__(256) void k_heavy_write(int n, const int* __restrict__ rp, const int* __restrict__ offsets,
                                                     int* __restrict__ heavy) {
    __shared__ int s_base;
    __shared__ int s_wave[256 / kWave];
    const int i0 = blockIdx.x * kHeavySpan;
    if (threadIdx.x == 0) s_base = offsets[blockIdx.x];
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / kWave;
    for (int c0 = i0; c0 < min(n, i0 + kHeavySpan); c0 += blockDim.x) {
        const int i = c0 + threadIdx.x;
        const bool h = i < min(n, i0 + kHeavySpan) && rp[i + 1] - rp[i] > kHeavyDegree;
        const uint64_t mask = __ballot(h);
        if (lane == 0) s_wave[w] = __popcll(mask);
        __syncthreads();
        int before = s_base;
        for (int q = 0; q < w; ++q) before += s_wave[q];
        if (h) heavy[before + mask_rank(mask)] = i;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int q = 0; q < (int)(blockDim.x / kWave); ++q) tot += s_wave[q];
            s_base += tot;
        }
        __syncthreads();
    }
}

ssm_status heavy_list(const ssm_csr* g, int** heavy, int32_t* count, hipStream_t s) {
    const int n = g->n;
    const int nb = div_up(n, kHeavySpan);
    *heavy = nullptr;
    *count = 0;
    int* buf = nullptr;  // counts[nb], total, ids[n]
    ssm_status st = salloc((void**)&buf, sizeof(int) * ((size_t)nb + 1 + n));
    if (st != SSM_OK) return st;
    int* counts = buf;
    int* total = buf + nb;
    int* ids = total + 1;
    hipLaunchKernelGGL(k_heavy_count, dim3(nb), dim3(256), 0, s, n, g->row_ptr, counts);
    hipLaunchKernelGGL(k_heavy_scan, dim3(1), dim3(64), 0, s, nb, counts, total);
    hipLaunchKernelGGL(k_heavy_write, dim3(nb), dim3(256), 0, s, n, g->row_ptr, counts, ids);
    hipError_t e = hipGetLastError();
    int nh = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&nh, total, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
        st = salloc((void**)heavy, sizeof(int) * (size_t)std::max(nh, 1));
        if (st != SSM_OK) {
            sfree(buf);  // the stream was synchronized above
            return st;
        }
        if (nh > 0) e = hipMemcpyAsync(*heavy, ids, sizeof(int) * (size_t)nh, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused (also after an error)
    sfree(buf);
    if (e != hipSuccess) {
        sfree(*heavy);  // the stream is idle
        *heavy = nullptr;
        return hip_fail(e, "heavy-node list");
    }
    *count = nh;
    return SSM_OK;
}

// ---------------------------------------- bit-parallel multi-source BFS

// One bit per pivot: vis[v][w] marks the pivots whose BFS has reached v,
// cur[v][w] those that reached v at the previous level.  Level L (bottom-up):
// every node ORs its neighbours' cur words, keeps the bits it has not seen
// and records dist[t][v] = L for each new bit t.  Efficient when the graph
// has few levels (hub-heavy graphs); the level loop runs on the host.
template <int NW>
__global__ __launch_bounds__(256) void k_msbfs_init(int n, int k, const int* __restrict__ pivots,
                                                   unsigned long long* __restrict__ vis,
                                                   unsigned long long* __restrict__ cur, int* __restrict__ dist) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k; t += gridDim.x * blockDim.x) {
        const int p = pivots[t];
        atomicOr(&vis[(size_t)p * NW + t / 64], 1ull << (t % 64));
        atomicOr(&cur[(size_t)p * NW + t / 64], 1ull << (t % 64));
        dist[(size_t)t * n + p] = 0;
    }
}

template <int NW>
__global__ __launch_bounds__(256) void k_msbfs_level(int n, int k, int level, const int* __restrict__ rp,
                                                    const int* __restrict__ ci,
                                                    unsigned long long* __restrict__ vis,
                                                    const unsigned long long* __restrict__ cur,
                                                    unsigned long long* __restrict__ nxt, int* __restrict__ dist,
                                                    unsigned long long* __restrict__ settled) {
    const int lane = lane_id();
    unsigned long long found = 0;
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int v = base + threadIdx.x;
        unsigned long long nw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) nw[w] = 0;
        if (v < n) {
            unsigned long long seen[NW], acc[NW];
            bool open = false;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int bits = min(64, k - 64 * w);
                const unsigned long long full = bits == 64 ? ~0ull : ((1ull << bits) - 1);
                seen[w] = vis[(size_t)v * NW + w];
                acc[w] = 0;
                open |= seen[w] != full;
            }
            if (open && rp[v + 1] - rp[v] > kHeavyDegree) open = false;  // k_msbfs_heavy's node
            if (open) {
                for (int e = rp[v]; e < rp[v + 1]; ++e) {
                    const int u = ci[e];
#pragma unroll
                    for (int w = 0; w < NW; ++w) acc[w] |= cur[(size_t)u * NW + w];
                }
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    nw[w] = acc[w] & ~seen[w];
                    if (nw[w]) vis[(size_t)v * NW + w] = seen[w] | nw[w];
                }
            }
            if (rp[v + 1] - rp[v] <= kHeavyDegree) {
#pragma unroll
                for (int w = 0; w < NW; ++w) nxt[(size_t)v * NW + w] = nw[w];
            }
        }
        // write distances pivot by pivot: loop over the bits set anywhere in
        // the wave, so lanes of a wave store consecutive nodes of one row
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            found += __popcll(nw[w]);
            unsigned long long wave_bits = nw[w];
            for (int off = 32; off > 0; off >>= 1) wave_bits |= __shfl_xor(wave_bits, off);
            while (wave_bits) {
                const int b = __ffsll(wave_bits) - 1;
                wave_bits &= wave_bits - 1;
                if ((nw[w] >> b) & 1ull) dist[(size_t)(64 * w + b) * n + v] = level;
            }
        }
    }
    found = wave_sum(found);
    if (found && lane == 0) atomicAdd(settled, found);
}

// The same level for the high-degree nodes, one wavefront per node: lanes
// OR strided slices of the neighbour list, a butterfly combines them.
template <int NW>
__global__ __launch_bounds__(256) void k_msbfs_heavy(int n, int k, int level, int nheavy,
                                                    const int* __restrict__ heavy, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, unsigned long long* __restrict__ vis,
                                                    const unsigned long long* __restrict__ cur,
                                                    unsigned long long* __restrict__ nxt, int* __restrict__ dist,
                                                    unsigned long long* __restrict__ settled) {
    const int lane = lane_id();
    unsigned long long found = 0;
    for (int h = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; h < nheavy;
         h += gridDim.x * blockDim.x / kWave) {
        const int v = heavy[h];
        unsigned long long seen[NW], acc[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            seen[w] = vis[(size_t)v * NW + w];
            acc[w] = 0;
        }
        for (int e = rp[v] + lane; e < rp[v + 1]; e += kWave) {
            const int u = ci[e];
#pragma unroll
            for (int w = 0; w < NW; ++w) acc[w] |= cur[(size_t)u * NW + w];
        }
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            for (int off = 32; off > 0; off >>= 1) acc[w] |= __shfl_xor(acc[w], off);
            const int bits = min(64, k - 64 * w);
            const unsigned long long full = bits == 64 ? ~0ull : ((1ull << bits) - 1);
            const unsigned long long nw = acc[w] & ~seen[w] & full;
            if (lane == 0) {
                nxt[(size_t)v * NW + w] = nw;
                if (nw) vis[(size_t)v * NW + w] = seen[w] | nw;
                found += __popcll(nw);
            }
            if ((nw >> lane) & 1ull) dist[(size_t)(64 * w + lane) * n + v] = level;
        }
    }
    found = wave_sum(found);
    if (found && lane == 0) atomicAdd(settled, found);
}

template <int NW>
static ssm_status msbfs(const ssm_csr* g, int32_t k, const int32_t* pivots, int32_t* dist, int budget,
                        bool forced, bool* done, int32_t* levels_out, hipStream_t s) {
    const int n = g->n;
    *done = false;
    unsigned long long* buf = nullptr;
    ssm_status st = salloc((void**)&buf, sizeof(unsigned long long) * (3 * (size_t)n * NW + 8));
    if (st != SSM_OK) return st;
    unsigned long long* vis = buf;
    unsigned long long* cur = vis + (size_t)n * NW;
    unsigned long long* nxt = cur + (size_t)n * NW;
    unsigned long long* settled = nxt + (size_t)n * NW;  // [0] this level, [1] all levels
    hipError_t e = hipMemsetAsync(buf, 0, sizeof(unsigned long long) * 2 * (size_t)n * NW, s);
    if (e == hipSuccess) e = hipMemsetAsync(dist, 0xff, sizeof(int) * (size_t)k * n, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_msbfs_init<NW>, dim3(div_up(k, 256)), dim3(256), 0, s, n, k, pivots, vis, cur, dist);
        e = hipGetLastError();
    }
    int* heavy = nullptr;
    int32_t nheavy = 0;
    if (e == hipSuccess) {
        st = heavy_list(g, &heavy, &nheavy, s);
        if (st != SSM_OK) {
            (void)hipStreamSynchronize(s);  // idle before the scratch is reused
            sfree(buf);
            return st;
        }
    }
    const int grid = std::min(div_up(n, 256), num_cus() * 8);
    const double pairs = (double)k * n;
    double total = k;  // the pivots themselves
    double prev = k;   // pairs settled at the previous level
    int level = 0;
    while (e == hipSuccess && level < budget) {
        ++level;
        unsigned long long h = 0;
        e = hipMemsetAsync(settled, 0, sizeof(unsigned long long), s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_msbfs_level<NW>, dim3(grid), dim3(256), 0, s, n, k, level, g->row_ptr, g->col_idx, vis,
                           cur, nxt, dist, settled);
        if (nheavy > 0)
            hipLaunchKernelGGL(k_msbfs_heavy<NW>, dim3(std::min(div_up(nheavy, 4), 4096)), dim3(256), 0, s, n, k,
                               level, nheavy, heavy, g->row_ptr, g->col_idx, vis, cur, nxt, dist, settled);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&h, settled, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        std::swap(cur, nxt);
        total += (double)h;
        if (h == 0) {
            *done = true;
            break;
        }
        // Every level is a pass over all nodes, so the form pays only when the
        // levels are few: on small-world graphs the pairs settled per level
        // multiply, on meshes and geometric graphs they grow by less than 2x
        // (d-dimensional balls), and those go to the per-pivot BFS after a
        // level or two.
        if (!forced && level >= 2 && total < 0.5 * pairs && (double)h < 2.0 * prev) break;
        prev = (double)h;
    }
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused
    sfree(buf);
    sfree(heavy);
    if (e != hipSuccess) return hip_fail(e, "bit-parallel BFS");
    *levels_out = level - 1;  // the last level found nothing
    return SSM_OK;
}

// Sum over nodes of the squared degree (one atomic per block).
__global__ __launch_bounds__(256) void k_degree_sq(int n, const int* __restrict__ rp, unsigned long long* out) {
    unsigned long long sq = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned long long d = (unsigned long long)(rp[i + 1] - rp[i]);
        sq += d * d;
    }
    __shared__ unsigned long long red[256 / kWave];
    sq = block_sum(sq, red);
    if (threadIdx.x == 0 && sq) atomicAdd(out, sq);
}

// Whether the bit-parallel BFS should go first: graphs with many arcs whose
// mean neighbour degree (sum d^2 / sum d) is at least kMsbfsSpread times the
// mean degree, i.e. hubs that most paths pass through, so the levels are
// few.  Measured on MI355X, rows and regions of 200 pivots: preferential-
// attachment graphs (ratio 3.3-4.1) of 1M nodes 18.8 -> 5.5 ms, 500k
// 8.7 -> 3.3 ms, 100k 2.0 -> 1.55 ms, 50k even; a 3.25M-node mesh (ratio
// 1.0) 37.5 -> 40.5 ms and a 100k random geometric graph (1.13) 1.5 ->
// 3.0 ms if forced, so those stay on the per-pivot BFS.
constexpr double kMsbfsSpread = 3.0;
constexpr long long kMsbfsMinArcs = 1LL << 19;

static ssm_status msbfs_pays(const ssm_csr* g, bool* pays, hipStream_t s) {
    *pays = false;
    if ((long long)g->nnz < kMsbfsMinArcs) return SSM_OK;
    unsigned long long* acc = nullptr;
    ssm_status st = salloc((void**)&acc, sizeof(unsigned long long));
    if (st != SSM_OK) return st;
    unsigned long long sq = 0;
    hipError_t e = hipMemsetAsync(acc, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_degree_sq, dim3(std::min(div_up(g->n, 256), 1024)), dim3(256), 0, s, g->n, g->row_ptr,
                           acc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&sq, acc, sizeof(sq), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused
    sfree(acc);
    if (e != hipSuccess) return hip_fail(e, "degree moments");
    const double arcs = (double)g->nnz, mean = arcs / (double)g->n;
    *pays = (double)sq / arcs >= kMsbfsSpread * mean;
    return SSM_OK;
}

// Checks every row of dist for an unreached node (-1); counts into *bad.
__global__ void k_count_unreached(long long total, const int* __restrict__ dist, int* bad) {
    int c = 0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x)
        c += dist[q] < 0;
    c = wave_sum(c);
    if (c && lane_id() == 0) atomicAdd(bad, c);
}

// ------------------------------------------------ padded adjacency (ELL)

// Row v of the padded adjacency holds the start of v's CSR row in W slots;
// unused slots hold -1.  A row longer than W keeps W - 1 entries and
// kEllMore in its last slot; the rest is read from the CSR row.  A frontier
// node's neighbours then arrive with one load that needs no row bounds.
constexpr int kEllMore = -2;

__global__ void k_ell_build(int n, int W, const int* __restrict__ rp, const int* __restrict__ ci,
                            int* __restrict__ ell) {
    const long long total = (long long)n * W;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int v = (int)(q / W), j = (int)(q - (long long)v * W);
        const int a = rp[v], d = rp[v + 1] - a;
        int val = -1;
        if (d > W && j == W - 1)
            val = kEllMore;
        else if (j < d)
            val = ci[a + j];
        ell[q] = val;
    }
}

// Slots per padded row: the mean degree rounded up to 8, 16 or 32.
static int ell_width(const ssm_csr* g) {
    const int forced = variant("ell_width");  // tuning override: 8, 16 or 32
    if (forced == 8 || forced == 16 || forced == 32) return forced;
    const double avg = g->n > 0 ? (double)g->nnz / g->n : 0.0;
    return avg <= 4.0 ? 8 : avg <= 12.0 ? 16 : 32;
}

static hipError_t ell_build(const ssm_csr* g, int W, int* ell, hipStream_t s) {
    const long long total = (long long)g->n * W;
    hipLaunchKernelGGL(k_ell_build, dim3(std::min(div_up(total, 256), 8192)), dim3(256), 0, s, g->n, W, g->row_ptr,
                       g->col_idx, ell);
    return hipGetLastError();
}

// ------------------------------------------------ LDS-resident BFS levels
//
// A workgroup runs a level-synchronous BFS whose visited set is one LDS bit
// per node: a neighbour is claimed by an LDS atomic OR, so the claiming lane
// owns the node for this BFS and writes its global state with plain stores.
// Frontiers are node ids: the first kLdsQ in LDS, the rest in a global
// overflow area of n entries.  Rows longer than W are listed (kHeavyCap in
// LDS, then global) and their CSR rest is read by whole waves after the
// regular part of the level.

constexpr int kLdsQ = 2048;
constexpr int kHeavyCap = 512;
constexpr int kLdsFixed = (2 * kLdsQ + kHeavyCap) * 4;  // LDS bytes besides the visited bits
constexpr int kBfsRows = 2;  // frontier nodes per lane group and pass in the per-pivot BFS

__host__ __device__ constexpr size_t lds_bits_bytes(long long n) { return (size_t)((n + 31) / 32) * 4; }

struct Frontier {
    const int* lcur;  // current frontier: LDS part, global part
    const int* gcur;
    int* lnxt;  // next frontier
    int* gnxt;
    int2* cnt;  // LDS counters of the level: x = long rows listed, y = size of the next frontier
    int* lheavy;  // long rows of the current frontier: LDS part, global part
    int* gheavy;
};

// Level counters rotate over three int2 slots: level l counts into slot
// l % 3, reads it once after its barrier and clears slot (l + 1) % 3 at its
// start (last read two levels earlier, a barrier ago), so one barrier and
// one LDS read per level suffice.
__device__ __forceinline__ void level_begin(int2* slots, int level, Frontier& f) {
    if (threadIdx.x == 0) slots[(level + 1) % 3] = make_int2(0, 0);
    f.cnt = &slots[level % 3];
}

// Entry i of a list split into an LDS part (first CAP entries) and a global
// part.  The explicit address spaces keep the two loads apart (a select of
// the two pointers would become one slower flat load).
template <int CAP>
__device__ __forceinline__ int split_get(const int* l, const int* g, int i) {
    if (i < CAP) return ((const __attribute__((address_space(3))) int*)l)[i];
    return ((const __attribute__((address_space(1))) int*)g)[i - CAP];
}


// Claims u[0..N) in the visited bits (one batch of LDS atomics); ok[j] is
// set where this lane claimed u[j] now.
template <int N>
__device__ __forceinline__ void claim(const int (&u)[N], bool (&ok)[N], unsigned* bits, int n) {
    unsigned old[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        ok[j] = (unsigned)u[j] < (unsigned)n;  // padding, continuation mark, bad index
        old[j] = ok[j] ? atomicOr(&bits[u[j] >> 5], 1u << (u[j] & 31)) : 0u;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) ok[j] = ok[j] && !(old[j] & (1u << (u[j] & 31)));
}

// Appends the u[j] with ok[j] to the next frontier: one reservation per wave.
// Call with every lane of the wave active.
template <int N>
__device__ __forceinline__ void append(const int (&u)[N], const bool (&ok)[N], const Frontier& f) {
    uint64_t mk[N];
    int tot = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        mk[j] = __ballot(ok[j]);
        tot += __popcll(mk[j]);
    }
    if (tot == 0) return;
    int at = 0;
    if (lane_id() == 0) at = atomicAdd(&f.cnt->y, tot);
    at = __builtin_amdgcn_readfirstlane(at);  // lane 0 is active: every lane is
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (ok[j]) {
            const int slot = at + mask_rank(mk[j]);
            if (slot < kLdsQ)
                f.lnxt[slot] = u[j];
            else
                f.gnxt[slot - kLdsQ] = u[j];
        }
        at += __popcll(mk[j]);
    }
}

// One level over the current frontier [0, len): each group of W/4 lanes takes
// P frontier nodes per pass (P row loads in flight per lane).
// take(u, ok) claims the neighbours u[j] (entries outside [0, n) are
// padding) and sets ok[j] for those that join the next frontier.  Ends with
// every thread past a barrier and the next frontier complete; returns its
// size.  Call from uniform control flow with blockDim.x a multiple of 64.
template <int W, int P, bool GLOBAL_PART, typename Take>
__device__ __forceinline__ void ell_passes(int n, const int* __restrict__ ell, int qbeg, int qend, const Frontier& f,
                                           Take& take) {
    constexpr int VW = W / 4;
    const int sub = threadIdx.x % VW, grp = threadIdx.x / VW, ngrp = blockDim.x / VW;
    const int wave_grp0 = __builtin_amdgcn_readfirstlane(grp - lane_id() / VW);  // first group of this wave
    for (int base = qbeg; base < qend; base += P * ngrp) {
        if (base + wave_grp0 >= qend) break;  // uniform per wave: no node of this pass (nor of later ones) here
        int4 nb[P];
        int v[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int qi = base + p * ngrp + grp;
            // the LDS part and the global part of the queue are walked by
            // separate passes: a register written by either a global or an
            // LDS load would make every LDS read wait for all outstanding
            // global stores
            if (GLOBAL_PART)
                v[p] = qi < qend ? ((const __attribute__((address_space(1))) int*)f.gcur)[qi - kLdsQ] : -1;
            else
                v[p] = qi < qend ? ((const __attribute__((address_space(3))) int*)f.lcur)[qi] : -1;
            nb[p] = make_int4(-1, -1, -1, -1);
            if ((unsigned)v[p] < (unsigned)n) nb[p] = *(const int4*)(ell + (size_t)v[p] * W + 4 * sub);
        }
        int u[4 * P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (sub == VW - 1 && nb[p].w == kEllMore) {
                const int h = atomicAdd(&f.cnt->x, 1);
                if (h < kHeavyCap)
                    f.lheavy[h] = v[p];
                else
                    f.gheavy[h - kHeavyCap] = v[p];
            }
            u[4 * p] = nb[p].x;
            u[4 * p + 1] = nb[p].y;
            u[4 * p + 2] = nb[p].z;
            u[4 * p + 3] = nb[p].w;
        }
        bool ok[4 * P];
        take(u, ok);
        append(u, ok, f);
    }
}

// One level over the current frontier [0, len): each group of W/4 lanes takes
// P frontier nodes per pass (P row loads in flight per lane).
// take(u, ok) claims the neighbours u[j] (entries outside [0, n) are
// padding) and sets ok[j] for those that join the next frontier.  Ends with
// every thread past a barrier and the next frontier complete; returns its
// size.  Call from uniform control flow with blockDim.x a multiple of 64.
template <int W, int P, typename Take>
__device__ __forceinline__ int ell_level(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                         const int* __restrict__ ell, int len, const Frontier& f, Take take) {
    static_assert(W / 4 >= 1 && W / 4 <= kWave && (kWave % (W / 4)) == 0, "lanes per node");
    ell_passes<W, P, false>(n, ell, 0, min(len, kLdsQ), f, take);
    if (len > kLdsQ) ell_passes<W, P, true>(n, ell, kLdsQ, len, f, take);  // uniform
    __syncthreads();
    const int2 c = *f.cnt;  // long rows, next frontier so far
    const int nh = min(c.x, n);
    if (nh > 0) {  // uniform
        const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave, lane = lane_id();
        for (int h = wave; h < nh; h += nwaves) {
            const int v = split_get<kHeavyCap>(f.lheavy, f.gheavy, h);
            const int e0 = rp[v] + W - 1, e1 = rp[v + 1];
            for (int e = e0; e < e1; e += 4 * kWave) {
                int u[4];
                bool ok[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ee = e + lane + j * kWave;
                    u[j] = ee < e1 ? ci[ee] : -1;
                }
                take(u, ok);
                append(u, ok, f);
            }
        }
        __syncthreads();
        return min(f.cnt->y, n);
    }
    return min(c.y, n);
}

// ell_level with P = 4 rows per lane group and pass for frontiers wider than
// one pass, P = 1 otherwise (uniform choice).
template <int W, typename Take>
__device__ __forceinline__ int ell_level_auto(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const int* __restrict__ ell, int len, const Frontier& f, Take take) {
    if (len > (int)blockDim.x / (W / 4)) return ell_level<W, 4>(n, rp, ci, ell, len, f, take);
    return ell_level<W, 1>(n, rp, ci, ell, len, f, take);
}

// Block b: BFS from pivots[b] writing dist[b][*] for every node it reaches,
// with the visited set in LDS bits.  gq holds 3 n ints per block (two
// frontier overflows, long-row overflow).  reached[b] = nodes found;
// *ecc_max = largest eccentricity seen.
// BFS from src writing D[*] for every node it reaches, with the visited set
// in LDS bits; gq holds 3 n ints (two frontier overflows, long-row
// overflow).  Thread 0 stores the number of nodes found in *reached and
// raises *ecc_max to the eccentricity of src.
template <int W, int POOL>
__device__ __forceinline__ void bfs_ell_body(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                             const int* __restrict__ ell, int src, int* D, int* gq, int* reached,
                                             int* ecc_max) {
    __shared__ __align__(16) unsigned char pool[POOL];
    __shared__ int2 s_slot[3];
    int* qa = (int*)pool;
    int* qb = qa + kLdsQ;
    int* lheavy = qb + kLdsQ;
    unsigned* bits = (unsigned*)(lheavy + kHeavyCap);
    int* ga = gq;
    int* gb = ga + n;
    int* gh = gb + n;
    const int nbw = (n + 31) / 32;
    for (int w = threadIdx.x; w < nbw; w += blockDim.x) bits[w] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        D[src] = 0;
        bits[src >> 5] |= 1u << (src & 31);
        qa[0] = src;
        s_slot[0] = make_int2(0, 0);
    }
    __syncthreads();
    Frontier f{qa, ga, qb, gb, nullptr, lheavy, gh};
    int level = 0, total = 1, len = 1;
    for (; len > 0; ++level) {
        level_begin(s_slot, level, f);
        const int dv = level + 1;
        len = ell_level_auto<W>(n, rp, ci, ell, len, f, [&](const auto& u, auto& ok) {
            constexpr int N = sizeof(u) / sizeof(u[0]);
            claim(u, ok, bits, n);
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (ok[j]) D[u[j]] = dv;
        });
        total += len;
        const int* tl = f.lcur;
        f.lcur = f.lnxt;
        f.lnxt = (int*)tl;
        const int* tg = f.gcur;
        f.gcur = f.gnxt;
        f.gnxt = (int*)tg;
    }
    if (threadIdx.x == 0) {
        *reached = total;
        atomicMax(ecc_max, level - 1);
    }
}

// Block b: BFS from pivots[b] into dist[b][*]; gq holds 3 n ints per block.
template <int W, int POOL>
__global__ __launch_bounds__(kBfsBlock) void k_bfs_ell(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const int* __restrict__ ell, const int* __restrict__ pivots,
                                                       int* dist, int* gq, int* reached, int* ecc_max) {
    const int b = blockIdx.x;
    bfs_ell_body<W, POOL>(n, rp, ci, ell, pivots[b], dist + (size_t)b * n, gq + (size_t)b * 3 * n, reached + b,
                          ecc_max);
}

// Block b: BFS from pivots[b] into dist[b][*] (pre-set to -1) for graphs
// whose visited bits do not fit in LDS: the padded adjacency and frontier
// queues of bfs_ell_body, the visited set being the distance row itself.  A
// neighbour is claimed by a compare-and-swap of its distance from -1 to the
// level (workgroup scope: the row belongs to this block), issued for all of
// a lane's neighbours before any result is used; with PRE, the distances are
// read first and only the unvisited ones are swapped.  gq holds 3 n ints per
// block.  reached[b] = nodes found; *ecc_max = largest eccentricity seen.
template <int W, bool PRE>
__global__ __launch_bounds__(kBfsBlock) void k_bfs_ell_g(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const int* __restrict__ ell,
                                                         const int* __restrict__ pivots, int* dist, int* gq,
                                                         int* reached, int* ecc_max) {
    __shared__ __align__(16) int pool[2 * kLdsQ + kHeavyCap];
    __shared__ int2 s_slot[3];
    const int b = blockIdx.x;
    int* D = dist + (size_t)b * n;
    int* qa = pool;
    int* qb = qa + kLdsQ;
    int* lheavy = qb + kLdsQ;
    int* ga = gq + (size_t)b * 3 * n;
    int* gb = ga + n;
    int* gh = gb + n;
    if (threadIdx.x == 0) {
        D[pivots[b]] = 0;
        qa[0] = pivots[b];
        s_slot[0] = make_int2(0, 0);
    }
    __syncthreads();
    Frontier f{qa, ga, qb, gb, nullptr, lheavy, gh};
    int level = 0, total = 1, len = 1;
    for (; len > 0; ++level) {
        level_begin(s_slot, level, f);
        const int dv = level + 1;
        len = ell_level_auto<W>(n, rp, ci, ell, len, f, [&](const auto& u, auto& ok) {
            constexpr int N = sizeof(u) / sizeof(u[0]);
            int old[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                ok[j] = (unsigned)u[j] < (unsigned)n;  // padding, continuation mark
                old[j] = PRE && ok[j] ? wg_load(&D[u[j]]) : -1;
            }
#pragma unroll
            for (int j = 0; j < N; ++j) {
                ok[j] = ok[j] && old[j] < 0;
                if (ok[j]) {
                    int expected = -1;
                    __hip_atomic_compare_exchange_strong(&D[u[j]], &expected, dv, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    old[j] = expected;
                }
            }
#pragma unroll
            for (int j = 0; j < N; ++j) ok[j] = ok[j] && old[j] == -1;
        });
        total += len;
        const int* tl = f.lcur;
        f.lcur = f.lnxt;
        f.lnxt = (int*)tl;
        const int* tg = f.gcur;
        f.gcur = f.gnxt;
        f.gnxt = (int*)tg;
    }
    if (threadIdx.x == 0) {
        reached[b] = total;
        atomicMax(ecc_max, level - 1);
    }
}

// LDS pool sizes of k_bfs_ell (several workgroups share a CU when small);
// 0 = the visited bits do not fit.
constexpr int kPoolS = 32768, kPoolM = 65536, kPoolL = 155648;

static int bfs_ell_pool(int n) {
    const size_t need = kLdsFixed + lds_bits_bytes(n);
    return need <= (size_t)kPoolS ? kPoolS : need <= (size_t)kPoolM ? kPoolM : need <= (size_t)kPoolL ? kPoolL : 0;
}

template <int W>
static hipError_t launch_bfs_ell_w(int pool, int blocks, hipStream_t s, int n, const int* rp, const int* ci,
                                   const int* ell, const int* pivots, int* dist, int* gq, int* reached, int* ecc) {
    if (pool == kPoolS)
        hipLaunchKernelGGL((k_bfs_ell<W, kPoolS>), dim3(blocks), dim3(kBfsBlock), 0, s, n, rp, ci, ell, pivots, dist,
                           gq, reached, ecc);
    else if (pool == kPoolM)
        hipLaunchKernelGGL((k_bfs_ell<W, kPoolM>), dim3(blocks), dim3(kBfsBlock), 0, s, n, rp, ci, ell, pivots, dist,
                           gq, reached, ecc);
    else
        hipLaunchKernelGGL((k_bfs_ell<W, kPoolL>), dim3(blocks), dim3(kBfsBlock), 0, s, n, rp, ci, ell, pivots, dist,
                           gq, reached, ecc);
    return hipGetLastError();
}

static hipError_t launch_bfs_ell(int W, int pool, int blocks, hipStream_t s, int n, const int* rp, const int* ci,
                                 const int* ell, const int* pivots, int* dist, int* gq, int* reached, int* ecc) {
    if (W == 8) return launch_bfs_ell_w<8>(pool, blocks, s, n, rp, ci, ell, pivots, dist, gq, reached, ecc);
    if (W == 16) return launch_bfs_ell_w<16>(pool, blocks, s, n, rp, ci, ell, pivots, dist, gq, reached, ecc);
    return launch_bfs_ell_w<32>(pool, blocks, s, n, rp, ci, ell, pivots, dist, gq, reached, ecc);
}

template <int VW>
static void launch_bfs_wg(int blocks, hipStream_t s, int n, const int* rp, const int* ci,
                          const int* pivots, int* dist, int2* queues, int* reached, int* ecc) {
    // Loads (LD of k_bfs_wg): plain CSR loads by default, measured on MI355X
    // for the 100 rows of a 3.25M-node mesh: 48 -> 44 ms (one row alone 44 ->
    // 36 ms); tuning: bfs_loads 2 = plain visited checks too, 3 = agent-scope
    // loads throughout.
    const int ld = variant("bfs_loads") == 3 ? 0 : variant("bfs_loads") == 2 ? 2 : 1;
    if (variant("bfs_rowq") == 2)          // tuning: node ids in the queue instead of row bounds
        hipLaunchKernelGGL((k_bfs_wg<VW, false, 0>), dim3(blocks), dim3(kBfsBlock), 0, s, n, rp, ci, pivots,
                           dist, queues, reached, ecc);
    else if (ld == 1)
        hipLaunchKernelGGL((k_bfs_wg<VW, true, 1>), dim3(blocks), dim3(kBfsBlock), 0, s, n, rp, ci, pivots,
                           dist, queues, reached, ecc);
    else if (ld == 2)
        hipLaunchKernelGGL((k_bfs_wg<VW, true, 2>), dim3(blocks), dim3(kBfsBlock), 0, s, n, rp, ci, pivots,
                           dist, queues, reached, ecc);
    else
        hipLaunchKernelGGL((k_bfs_wg<VW, true, 0>), dim3(blocks), dim3(kBfsBlock), 0, s, n, rp, ci, pivots,
                           dist, queues, reached, ecc);
}

// Rows on kBfsGrp workgroups each (k_bfs_grp, defined below).
constexpr int kBfsGrp = 2;
hipError_t launch_bfs_grp(int vw, int rows, hipStream_t s, int n, const int* rp, const int* ci, const int* pivots,
                          int* dist, int2* queues, int* ctl, unsigned long long* bars, int* reached, int* ecc,
                          int* status);
int bfs_grp_fits(int rows);

ssm_status mssp(const ssm_csr* g, int32_t k, const int32_t* pivots, int32_t* dist,
                int32_t* dmax_out_host, hipStream_t s) {
    const int n = g->n;
    // Bit-parallel BFS over all pivots at once on large hub-dominated graphs
    // (msbfs_pays).  It hands over to the per-pivot BFS below when the
    // settled pairs stop multiplying, or after `budget` levels.  (tuning:
    // msbfs -1 = never, 1 = always, with no hand-over but the budget)
    const int budget = variant("msbfs_budget") > 0 ? variant("msbfs_budget") : 24;
    const int ms = variant("msbfs");
    bool use_ms = k <= 1024 && ms == 1;
    if (k <= 1024 && ms == 0) {
        ssm_status st = msbfs_pays(g, &use_ms, s);
        if (st != SSM_OK) return st;
    }
    if (use_ms) {
        bool done = false;
        int32_t levels = 0;
        ssm_status st;
        const int nw = div_up(k, 64);
        const bool forced = ms == 1;
        if (nw <= 1) st = msbfs<1>(g, k, pivots, dist, budget, forced, &done, &levels, s);
        else if (nw <= 2) st = msbfs<2>(g, k, pivots, dist, budget, forced, &done, &levels, s);
        else if (nw <= 4) st = msbfs<4>(g, k, pivots, dist, budget, forced, &done, &levels, s);
        else if (nw <= 8) st = msbfs<8>(g, k, pivots, dist, budget, forced, &done, &levels, s);
        else st = msbfs<16>(g, k, pivots, dist, budget, forced, &done, &levels, s);
        // chosen by the library, the form gives way to the per-pivot BFS when
        // its bit arrays do not fit
        if (st == SSM_E_NOMEM && !forced) done = false;
        else if (st != SSM_OK) return st;
        if (done) {
            int* bad = nullptr;
            st = salloc((void**)&bad, sizeof(int));
            if (st != SSM_OK) return st;
            int hbad = 0;
            hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
            if (e == hipSuccess) {
                long long total = (long long)k * n;
                hipLaunchKernelGGL(k_count_unreached, dim3((int)std::min<long long>((total + 255) / 256, 4096)),
                                   dim3(256), 0, s, total, dist, bad);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            (void)hipStreamSynchronize(s);
            sfree(bad);
            if (e != hipSuccess) return hip_fail(e, "bit-parallel BFS check");
            if (hbad) return fail(SSM_E_DISCONNECTED, "graph is not connected (a BFS missed nodes)");
            *dmax_out_host = levels;
            return SSM_OK;
        }
    }
    // LDS-resident BFS per pivot when the visited bits fit in LDS (tuning
    // override SSM_BFS_ELL=2 keeps the global-memory form).
    const int pool = bfs_ell_pool(n);
    if (pool > 0 && variant("bfs_ell") != 2 && variant("bfs_ell") != 3 && variant("bfs_ell") != 4) {
        const int W = ell_width(g);
        const long long qcap = 1LL << 31;  // overflow ints (8 GiB)
        const int batch = (int)std::max<long long>(1, std::min<long long>(k, qcap / (3LL * n)));
        int* ell = nullptr;
        int* gq = nullptr;
        int* aux = nullptr;  // reached[k], ecc
        ssm_status st = salloc((void**)&ell, sizeof(int) * (size_t)n * W);
        if (st == SSM_OK) st = salloc((void**)&gq, sizeof(int) * 3 * (size_t)n * batch);
        if (st == SSM_OK) st = salloc((void**)&aux, sizeof(int) * ((size_t)k + 1));
        hipError_t e = hipSuccess;
        std::vector<int> host((size_t)k + 1);
        if (st == SSM_OK) {
            e = hipMemsetAsync(aux, 0, sizeof(int) * ((size_t)k + 1), s);
            if (e == hipSuccess) e = ell_build(g, W, ell, s);
            for (int b0 = 0; b0 < k && e == hipSuccess; b0 += batch) {
                const int nb = std::min(batch, k - b0);
                e = launch_bfs_ell(W, pool, nb, s, n, g->row_ptr, g->col_idx, ell, pivots + b0,
                                   dist + (size_t)b0 * n, gq, aux + b0, aux + k);
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(host.data(), aux, sizeof(int) * ((size_t)k + 1), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        (void)hipStreamSynchronize(s);  // idle before the scratch is reused
        if (ell) sfree(ell);
        if (gq) sfree(gq);
        if (aux) sfree(aux);
        if (st != SSM_OK) return st;
        if (e != hipSuccess) return hip_fail(e, "multi-source BFS");
        for (int t = 0; t < k; ++t)
            if (host[t] != n) return fail(SSM_E_DISCONNECTED, "graph is not connected (a BFS missed nodes)");
        *dmax_out_host = host[k];
        return SSM_OK;
    }
    // Too large for LDS visited bits: variant bfs_ell = 3 (or 4: without the
    // read before the swap) takes the same padded-adjacency BFS with the
    // distance row as visited set; the default is the CSR form below (faster
    // on a 3.25M-node mesh: 57 against 84 ms for 100 rows without the read).
    if (variant("bfs_ell") == 3 || variant("bfs_ell") == 4) {
        const int W = ell_width(g);
        const long long qcap = 1LL << 31;  // overflow ints (8 GiB)
        const int batch = (int)std::max<long long>(1, std::min<long long>(k, qcap / (3LL * n)));
        int* ell = nullptr;
        int* gq = nullptr;
        int* aux = nullptr;  // reached[k], ecc
        ssm_status st = salloc((void**)&ell, sizeof(int) * (size_t)n * W);
        if (st == SSM_OK) st = salloc((void**)&gq, sizeof(int) * 3 * (size_t)n * batch);
        if (st == SSM_OK) st = salloc((void**)&aux, sizeof(int) * ((size_t)k + 1));
        hipError_t e = hipSuccess;
        std::vector<int> host((size_t)k + 1);
        if (st == SSM_OK) {
            e = hipMemsetAsync(dist, 0xff, sizeof(int) * (size_t)k * n, s);
            if (e == hipSuccess) e = hipMemsetAsync(aux, 0, sizeof(int) * ((size_t)k + 1), s);
            if (e == hipSuccess) e = ell_build(g, W, ell, s);
            for (int b0 = 0; b0 < k && e == hipSuccess; b0 += batch) {
                const int nb = std::min(batch, k - b0);
                const bool pre = variant("bfs_ell") != 4;
                auto kern = W == 8 ? (pre ? k_bfs_ell_g<8, true> : k_bfs_ell_g<8, false>)
                          : W == 16 ? (pre ? k_bfs_ell_g<16, true> : k_bfs_ell_g<16, false>)
                                    : (pre ? k_bfs_ell_g<32, true> : k_bfs_ell_g<32, false>);
                hipLaunchKernelGGL(kern, dim3(nb), dim3(kBfsBlock), 0, s, n, g->row_ptr, g->col_idx, ell,
                                   pivots + b0, dist + (size_t)b0 * n, gq, aux + b0, aux + k);
                e = hipGetLastError();
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(host.data(), aux, sizeof(int) * ((size_t)k + 1), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        (void)hipStreamSynchronize(s);  // idle before the scratch is reused
        if (ell) sfree(ell);
        if (gq) sfree(gq);
        if (aux) sfree(aux);
        if (st != SSM_OK) return st;
        if (e != hipSuccess) return hip_fail(e, "multi-source BFS");
        for (int t = 0; t < k; ++t)
            if (host[t] != n) return fail(SSM_E_DISCONNECTED, "graph is not connected (a BFS missed nodes)");
        *dmax_out_host = host[k];
        return SSM_OK;
    }
    // Sources run in batches so that the frontier queues stay bounded (every
    // queue entry is written before it is read: no clearing).
    const long long qcap = 1LL << 31;  // queue entries (16 GiB)
    int batch = (int)std::max<long long>(1, std::min<long long>(k, qcap / (2LL * n)));
    int2* queues = nullptr;
    int* aux = nullptr;  // reached[k], ecc
    ssm_status st = salloc((void**)&queues, sizeof(int2) * 2 * (size_t)n * batch);
    if (st != SSM_OK) return st;
    st = salloc((void**)&aux, sizeof(int) * ((size_t)k + 1));
    if (st != SSM_OK) {
        sfree(queues);
        return st;
    }
    hipError_t e = hipMemsetAsync(dist, 0xff, sizeof(int) * (size_t)k * n, s);
    if (e == hipSuccess) e = hipMemsetAsync(aux, 0, sizeof(int) * ((size_t)k + 1), s);
    int vw = virtual_warp(g);
    // kBfsGrp workgroups per row when every row's blocks get CUs of their own
    // (measured on MI355X: the 100 rows of a 3.25M-node mesh 44 -> 36 ms, its
    // slowest row alone 40 -> 29 ms; tuning: bfs_grp -1 = one workgroup)
    const bool grp = variant("bfs_grp") != -1 && (long long)batch * kBfsGrp <= num_cus() && bfs_grp_fits(batch);
    int* gctl = nullptr;  // per row: 32 ints (frontier counters), then 16 u64 (barrier) per row, then status
    if (grp && e == hipSuccess) {
        st = salloc((void**)&gctl, sizeof(int) * (size_t)batch * 32 + sizeof(unsigned long long) * (size_t)batch * 16 + 256);
        if (st != SSM_OK) {
            (void)hipStreamSynchronize(s);
            sfree(queues);
            sfree(aux);
            return st;
        }
    }
    int hstatus = 0;
    for (int b0 = 0; b0 < k && e == hipSuccess; b0 += batch) {
        int nb = std::min(batch, k - b0);
        int* D = dist + (size_t)b0 * n;
        int* reached = aux + b0;
        int* ecc = aux + k;
        if (grp) {
            unsigned long long* gbars = (unsigned long long*)(gctl + (size_t)batch * 32);
            int* gstatus = (int*)(gbars + (size_t)batch * 16);
            e = hipMemsetAsync(gbars, 0, sizeof(unsigned long long) * (size_t)batch * 16 + 256, s);
            if (e == hipSuccess)
                e = launch_bfs_grp(vw, nb, s, n, g->row_ptr, g->col_idx, pivots + b0, D, queues, gctl, gbars, reached,
                                   ecc, gstatus);
            if (e == hipSuccess) e = hipMemcpyAsync(&hstatus, gstatus, sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess && hstatus) break;
            continue;
        }
        switch (vw) {
            case 2: launch_bfs_wg<2>(nb, s, n, g->row_ptr, g->col_idx, pivots + b0, D, queues, reached, ecc); break;
            case 4: launch_bfs_wg<4>(nb, s, n, g->row_ptr, g->col_idx, pivots + b0, D, queues, reached, ecc); break;
            case 8: launch_bfs_wg<8>(nb, s, n, g->row_ptr, g->col_idx, pivots + b0, D, queues, reached, ecc); break;
            case 16: launch_bfs_wg<16>(nb, s, n, g->row_ptr, g->col_idx, pivots + b0, D, queues, reached, ecc); break;
            case 32: launch_bfs_wg<32>(nb, s, n, g->row_ptr, g->col_idx, pivots + b0, D, queues, reached, ecc); break;
            default: launch_bfs_wg<64>(nb, s, n, g->row_ptr, g->col_idx, pivots + b0, D, queues, reached, ecc); break;
        }
        e = hipGetLastError();
    }
    std::vector<int> host((size_t)k + 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), aux, sizeof(int) * ((size_t)k + 1), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused (also after an error)
    sfree(queues);
    sfree(aux);
    if (gctl) sfree(gctl);
    if (e != hipSuccess) return hip_fail(e, "multi-source BFS");
    if (hstatus) return fail(SSM_E_DEVICE, "multi-source BFS: a row's barrier did not fill and was aborted");
    for (int t = 0; t < k; ++t)
        if (host[t] != n) return fail(SSM_E_DISCONNECTED, "graph is not connected (a BFS missed nodes)");
    *dmax_out_host = host[k];
    return SSM_OK;
}

// ------------------------------------------------- max/min pivot sampling

__device__ __forceinline__ void grid_barrier(cg::grid_group& grid) {
    if (gridDim.x == 1)
        __syncthreads();
    else
        grid.sync();
}

// Largest of keys[0 .. count-1] for a whole wave (agent-scope loads, one per
// lane and pass, then a butterfly); every lane gets it.
__device__ __forceinline__ unsigned long long keys_max(const unsigned long long* keys, int count) {
    unsigned long long b = 0;
    for (int q = lane_id(); q < count; q += kWave) {
        const unsigned long long kq = __hip_atomic_load(&keys[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b = kq > b ? kq : b;
    }
    return wave_max(b);
}

// One launch per pivot t.  BFS from pivots[t] that only continues through
// nodes whose distance to the new pivot is smaller than m (their distance to
// the nearest earlier pivot), updating m on the way.  This is exact for
// m <- min(m, d_t): m is 1-Lipschitz along edges, so a node with d_t >= m
// cannot lead to a node where d_t < m.  Then pivots[t+1] = argmax m, lowest
// id on ties.  ctl[0..2] rotate as frontier counters; keys holds one partial
// argmax per block.  status[0] is set to 1 if the first BFS misses a node.
template <int VW>
__global__ __launch_bounds__(kSelBlock) void k_select(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, int t, int k,
                                                      int first, int* pivots, int* m, int* vis,
                                                      int* qa, int* qb, int* ctl,
                                                      unsigned long long* keys, int* status) {
    cg::grid_group grid = cg::this_grid();
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    const int src = (t == 0) ? first : pivots[t];
    if (gtid == 0) {
        if (t == 0) pivots[0] = first;
        vis[src] = t;
        m[src] = 0;
        qa[0] = src;
        ctl[0] = 1;
        ctl[1] = 0;
        ctl[2] = 0;
    }
    grid_barrier(grid);
    const int sub = gtid % VW, grp = gtid / VW, ngrp = nthreads / VW;
    int level = 0;
    int* cur = qa;
    int* nxt = qb;
    for (;;) {
        const int len = min(load_agent(&ctl[level % 3]), n);
        if (len == 0) break;
        int* tail = &ctl[(level + 1) % 3];
        if (gtid == 0) ctl[(level + 2) % 3] = 0;
        const int dv = level + 1;
        for (int base = 0; base < len; base += ngrp) {
            int qi = base + grp;
            int e0 = 0, e1 = 0;
            if (qi < len) {
                int u = cur[qi];
                if ((unsigned)u < (unsigned)n) {
                    e0 = rp[u];
                    e1 = rp[u + 1];
                }
            }
            for (int e = e0 + sub; e < e1; e += VW) {
                int v = ci[e];
                bool push = false;
                if (vis[v] != t && atomicExch(&vis[v], t) != t) {
                    if (dv < m[v]) {
                        m[v] = dv;
                        push = true;
                    }
                }
                int slot = wave_append(push, tail);
                if (push) nxt[slot] = v;
            }
        }
        grid_barrier(grid);
        int* tmp = cur;
        cur = nxt;
        nxt = tmp;
        ++level;
    }
    if (t + 1 >= k && t != 0) return;
    // argmax of m, lowest id on ties: maximize (m << 32) | ~id
    unsigned long long best = 0;
    for (int i = gtid; i < n; i += nthreads) {
        unsigned long long key =
            ((unsigned long long)(unsigned)m[i] << 32) | (unsigned long long)(0xffffffffu - (unsigned)i);
        best = key > best ? key : best;
    }
    __shared__ unsigned long long s_red[kSelBlock / kWave];
    best = block_max(best, s_red);
    if (threadIdx.x == 0) keys[blockIdx.x] = best;
    grid_barrier(grid);
    if (blockIdx.x == 0 && threadIdx.x < kWave) {  // wave 0 reads the keys, one per lane
        const unsigned long long b = keys_max(keys, (int)gridDim.x);
        if (threadIdx.x == 0) {
            int mbest = (int)(b >> 32);
            if (t == 0 && mbest == kInf) status[0] = 1;
            if (t + 1 < k) pivots[t + 1] = (int)(0xffffffffu - (unsigned)(b & 0xffffffffu));
        }
    }
}

// All k pivots in one cooperative launch.  For each t: BFS from pivots[t]
// that continues only through nodes whose distance to the new pivot is below
// m (their distance to the nearest earlier pivot): a relaxation lowers m with
// one atomicMin and the node joins the next frontier iff the atomic lowered
// it.  This is exact for m <- min(m, d_t) because m is 1-Lipschitz along
// edges (a node with d_t >= m cannot lead to a node where d_t < m).  Then
// pivots[t+1] = argmax m, lowest id on ties.  m is pre-set to INT_MAX.
template <int VW>
__global__ __launch_bounds__(kSelBlock) void k_select_all(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci, int k, int first,
                                                          int* pivots, int* m, int* qa, int* qb, int* ctl,
                                                          unsigned long long* keys, int* status) {
    cg::grid_group grid = cg::this_grid();
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    const int sub = gtid % VW, grp = gtid / VW, ngrp = nthreads / VW;
    __shared__ unsigned long long s_red[kSelBlock / kWave];
    for (int t = 0; t < k; ++t) {
        const int src = (t == 0) ? first : load_agent(&pivots[t]);
        if (gtid == 0) {
            if (t == 0) pivots[0] = first;
            m[src] = 0;
            qa[0] = src;
            ctl[0] = 1;
            ctl[1] = 0;
            ctl[2] = 0;
        }
        grid_barrier(grid);
        int level = 0;
        int* cur = qa;
        int* nxt = qb;
        for (;;) {
            const int len = min(load_agent(&ctl[level % 3]), n);
            if (len == 0) break;
            int* tail = &ctl[(level + 1) % 3];
            if (gtid == 0) ctl[(level + 2) % 3] = 0;
            const int dv = level + 1;
            for (int base = 0; base < len; base += ngrp) {
                int qi = base + grp;
                int e0 = 0, e1 = 0;
                if (qi < len) {
                    int u = cur[qi];
                    if ((unsigned)u < (unsigned)n) {
                        e0 = rp[u];
                        e1 = rp[u + 1];
                    }
                }
                for (int e = e0 + sub; e < e1; e += VW) {
                    int v = ci[e];
                    bool push = false;
                    if (m[v] > dv) push = atomicMin(&m[v], dv) > dv;  // stale reads are only larger
                    int slot = wave_append(push, tail);
                    if (push) nxt[slot] = v;
                }
            }
            grid_barrier(grid);
            int* tmp = cur;
            cur = nxt;
            nxt = tmp;
            ++level;
        }
        if (t + 1 >= k && t != 0) break;
        unsigned long long best = 0;
        for (int i = gtid; i < n; i += nthreads) {
            unsigned long long key =
                ((unsigned long long)(unsigned)m[i] << 32) | (unsigned long long)(0xffffffffu - (unsigned)i);
            best = key > best ? key : best;
        }
        best = block_max(best, s_red);
        if (threadIdx.x == 0) keys[blockIdx.x] = best;
        grid_barrier(grid);
        if (blockIdx.x == 0 && threadIdx.x < kWave) {  // wave 0 reads the keys, one per lane
            const unsigned long long b = keys_max(keys, (int)gridDim.x);
            if (threadIdx.x == 0) {
                if (t == 0 && (int)(b >> 32) == kInf) status[0] = 1;
                if (t + 1 < k) pivots[t + 1] = (int)(0xffffffffu - (unsigned)(b & 0xffffffffu));
            }
        }
        grid_barrier(grid);
        if (t == 0 && load_agent(&status[0]) != 0) break;  // disconnected: stop (uniform)
    }
}

// Key of node i with value m for the argmax: the largest m wins, then the
// lowest id.
__device__ __forceinline__ unsigned long long argmax_key(int m, int i) {
    return ((unsigned long long)(unsigned)m << 32) | (unsigned long long)(0xffffffffu - (unsigned)i);
}

__device__ __forceinline__ unsigned long long key_max(unsigned long long a, unsigned long long b) {
    return a > b ? a : b;
}

// Frontiers up to this size lower m with the atomic alone; wider ones read m
// first and skip the atomic where m is already at most the new distance.
constexpr int kSelPrecheck = 16384;

// Agent-scope accesses for data that blocks of one launch exchange: relaxed
// atomic loads and stores compile to cache-bypassing (sc1) accesses, so what
// one block stored and waited for is what another block loads, with no cache
// writeback or invalidation between them.
__device__ __forceinline__ void store_agent(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int4 load_agent4(const int* p) {  // p 16-byte aligned
    unsigned long long* q = (unsigned long long*)p;
    const unsigned long long a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_int4((int)(unsigned)a, (int)(unsigned)(a >> 32), (int)(unsigned)b, (int)(unsigned)(b >> 32));
}

// Grid barrier of a cooperative launch whose blocks share data only through
// agent-scope atomics and the agent-scope loads and stores above: every
// thread waits for its own memory operations to complete, then one thread
// per block counts in on a 64-bit counter and polls it until the whole grid
// has arrived (about 1.4 us for 32 blocks on MI355X against 4.6 us for the
// cooperative-groups grid sync, whose cache writeback and invalidation this
// sharing does not need).  bar is zeroed before the launch and serves one
// launch; epoch (thread 0's) is the count that ends the current barrier.  A
// barrier still not full after 2^25 polls (seconds) sets the counter's top
// bit, which every block sees on its next poll: sync_grid then returns false
// in every block and the kernel leaves, so a broken count ends in an error
// rather than a hang.
constexpr unsigned long long kBarAbort = 1ull << 63;
constexpr long long kBarPolls = 1ll << 25;

__device__ __forceinline__ bool sync_count(unsigned long long* bar, unsigned long long& epoch, int blocks) {
    __shared__ int s_go;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        epoch += blocks;
        unsigned long long v = __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        long long polls = 0;
        while ((v & kBarAbort) == 0 && (long long)(v - epoch) < 0) {
            if (++polls > kBarPolls) {
                v = __hip_atomic_fetch_or(bar, kBarAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) | kBarAbort;
                break;
            }
            v = __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_go = (v & kBarAbort) == 0;
    }
    __syncthreads();
    return s_go != 0;
}

// The barrier over the whole grid (see sync_count).
__device__ __forceinline__ bool sync_grid(unsigned long long* bar, unsigned long long& epoch) {
    return sync_count(bar, epoch, gridDim.x);
}

// Appends the u[j] with ok[j] (j < 4) to a global frontier with agent-scope
// stores: one counter reservation per wave.  Call with every lane active.
__device__ __forceinline__ void append4_agent(const int (&u)[4], const bool (&ok)[4], int* tail, int* nxt) {
    uint64_t mk[4];
    int tot = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        mk[j] = __ballot(ok[j]);
        tot += __popcll(mk[j]);
    }
    if (tot == 0) return;
    int at = 0;
    if (lane_id() == 0) at = atomicAdd(tail, tot);
    at = __builtin_amdgcn_readfirstlane(at);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (ok[j]) store_agent(&nxt[at + mask_rank(mk[j])], u[j]);
        at += __popcll(mk[j]);
    }
}

// ---------------------------------------- one BFS per kBfsGrp workgroups

// Rows on kBfsGrp workgroups each (cooperative launch, blocks g*kBfsGrp ..
// g*kBfsGrp + kBfsGrp - 1 for source g): the level-synchronous BFS of
// k_bfs_wg, its frontier (row bounds, as there) shared by the row's blocks
// through agent-scope loads and stores in the global queues, a claim by an
// agent-scope compare-and-swap on the distance, one reservation per wave on
// the row's frontier counter (ctl + 32 g: three level slots) and a barrier
// of the row's blocks per level (bars + 16 g).  A barrier that never fills
// sets status[0] and both blocks leave.

__device__ __forceinline__ int2 load_agent_int2(const int2* p) {
    const unsigned long long v =
        __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_int2((int)(unsigned)v, (int)(unsigned)(v >> 32));
}

__device__ __forceinline__ void store_agent_int2(int2* p, int2 v) {
    store_agent((unsigned long long*)p, (unsigned long long)(unsigned)v.x | ((unsigned long long)(unsigned)v.y << 32));
}

template <int VW>
__global__ __launch_bounds__(kBfsBlock) void k_bfs_grp(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const int* __restrict__ pivots, int* dist, int2* queues,
                                                       int* ctl, unsigned long long* bars, int* reached,
                                                       int* ecc_max, int* status) {
    const int g = blockIdx.x / kBfsGrp, part = blockIdx.x % kBfsGrp;
    int* D = dist + (size_t)g * n;
    int2* cur = queues + (size_t)g * 2 * n;
    int2* nxt = cur + n;
    int* c = ctl + 32 * g;
    unsigned long long* bar = bars + 16 * g;
    __shared__ int s_found;
    unsigned long long epoch = 0;
    const int src = pivots[g];
    if (threadIdx.x == 0) s_found = 0;
    if (part == 0 && threadIdx.x == 0) {
        store_agent(&D[src], 0);
        store_agent_int2(&cur[0], make_int2(rp[src], rp[src + 1]));
        store_agent(&c[0], 1);
        store_agent(&c[1], 0);
        store_agent(&c[2], 0);
    }
    if (!sync_count(bar, epoch, kBfsGrp)) {
        if (threadIdx.x == 0) store_agent(&status[0], 1);
        return;
    }
    const int sub = threadIdx.x % VW, grp = threadIdx.x / VW, ngrp = blockDim.x / VW;
    const int gg = part * ngrp + grp, ngg = kBfsGrp * ngrp;  // this lane group among the row's groups
    int level = 0;
    for (;;) {
        const int len = min(load_agent(&c[level % 3]), n);
        if (len == 0) break;
        int* tail = &c[(level + 1) % 3];
        if (part == 0 && threadIdx.x == 0) store_agent(&c[(level + 2) % 3], 0);
        for (int base = 0; base < len; base += ngg * kBfsU) {
            int2 row[kBfsU];
            int span = 0;
#pragma unroll
            for (int q = 0; q < kBfsU; ++q) {
                const int qi = base + q * ngg + gg;
                row[q] = qi < len ? load_agent_int2(&cur[qi]) : make_int2(0, 0);
                span = max(span, row[q].y - row[q].x);
            }
            for (int j = sub; j < span; j += VW) {
                int v[kBfsU], seen[kBfsU];
#pragma unroll
                for (int q = 0; q < kBfsU; ++q) v[q] = row[q].x + j < row[q].y ? ci[row[q].x + j] : -1;
#pragma unroll
                for (int q = 0; q < kBfsU; ++q) seen[q] = (unsigned)v[q] < (unsigned)n ? load_agent(&D[v[q]]) : 0;
                bool claim[kBfsU];
#pragma unroll
                for (int q = 0; q < kBfsU; ++q) {
                    claim[q] = false;
                    if ((unsigned)v[q] < (unsigned)n && seen[q] < 0) {
                        int expected = -1;
                        claim[q] = __hip_atomic_compare_exchange_strong(&D[v[q]], &expected, level + 1,
                                                                        __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                int2 vrow[kBfsU];
#pragma unroll
                for (int q = 0; q < kBfsU; ++q)
                    if (claim[q]) vrow[q] = make_int2(rp[v[q]], rp[v[q] + 1]);
                uint64_t mk[kBfsU];
                int tot = 0;
#pragma unroll
                for (int q = 0; q < kBfsU; ++q) {
                    mk[q] = __ballot(claim[q]);
                    tot += __popcll(mk[q]);
                }
                if (tot > 0) {  // uniform over the wave's active lanes
                    // the lowest active lane reserves (lane groups leave this
                    // loop at different times: rows of different lengths)
                    const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;
                    int at = 0;
                    if (lane_id() == leader) {
                        at = atomicAdd(tail, tot);
                        atomicAdd(&s_found, tot);
                    }
                    at = __shfl(at, leader);
#pragma unroll
                    for (int q = 0; q < kBfsU; ++q) {
                        if (claim[q]) store_agent_int2(&nxt[at + mask_rank(mk[q])], vrow[q]);
                        at += __popcll(mk[q]);
                    }
                }
            }
        }
        if (!sync_count(bar, epoch, kBfsGrp)) {
            if (threadIdx.x == 0) store_agent(&status[0], 1);
            return;
        }
        int2* t0 = cur;
        cur = nxt;
        nxt = t0;
        ++level;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&reached[g], s_found + (part == 0 ? 1 : 0));
        if (part == 0) atomicMax(ecc_max, level - 1);
    }
}

template <int VW>
static hipError_t launch_bfs_grp_w(int rows, hipStream_t s, int n, const int* rp, const int* ci, const int* pivots,
                                   int* dist, int2* queues, int* ctl, unsigned long long* bars, int* reached,
                                   int* ecc, int* status) {
    void* args[] = {&n, &rp, &ci, &pivots, &dist, &queues, &ctl, &bars, &reached, &ecc, &status};
    return hipLaunchCooperativeKernel((const void*)k_bfs_grp<VW>, dim3(rows * kBfsGrp), dim3(kBfsBlock), args, 0, s);
}

hipError_t launch_bfs_grp(int vw, int rows, hipStream_t s, int n, const int* rp, const int* ci, const int* pivots,
                          int* dist, int2* queues, int* ctl, unsigned long long* bars, int* reached, int* ecc,
                          int* status) {
    switch (vw) {
        case 2: return launch_bfs_grp_w<2>(rows, s, n, rp, ci, pivots, dist, queues, ctl, bars, reached, ecc, status);
        case 4: return launch_bfs_grp_w<4>(rows, s, n, rp, ci, pivots, dist, queues, ctl, bars, reached, ecc, status);
        case 8: return launch_bfs_grp_w<8>(rows, s, n, rp, ci, pivots, dist, queues, ctl, bars, reached, ecc, status);
        case 16: return launch_bfs_grp_w<16>(rows, s, n, rp, ci, pivots, dist, queues, ctl, bars, reached, ecc, status);
        case 32: return launch_bfs_grp_w<32>(rows, s, n, rp, ci, pivots, dist, queues, ctl, bars, reached, ecc, status);
        default: return launch_bfs_grp_w<64>(rows, s, n, rp, ci, pivots, dist, queues, ctl, bars, reached, ecc, status);
    }
}

// Whether rows x kBfsGrp blocks of k_bfs_grp are resident at once.
int bfs_grp_fits(int rows) {
    int a = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void*)k_bfs_grp<8>, kBfsBlock, 0) != hipSuccess)
        return 0;
    return (long long)rows * kBfsGrp <= (long long)a * num_cus();
}

// Pivots t0 .. t1-1 of max/min sampling in one cooperative launch, over the
// padded adjacency: each group of W/4 lanes takes one frontier node and four
// of its neighbours per lane (a longer row's CSR tail is walked by the same
// lanes).  The pruned BFS and the argmax are those of k_select_all: a
// relaxation lowers m with one atomicMin and the node joins the next frontier
// iff the atomic lowered it.  Blocks share the frontiers, counters, m and the
// partial keys through agent-scope accesses only, so the levels end in
// sync_grid.  The argmax reads m 16 bytes at a time, four in flight per
// thread (lowest id on ties through the key).  status[1] = the largest m
// after pivot 0's BFS (its eccentricity); status[2] = 1 if a grid barrier
// aborted.
template <int W>
__global__ __launch_bounds__(kSelBlock) void k_select_grid(int n, const int* __restrict__ rp,
                                                           const int* __restrict__ ci, const int* __restrict__ ell,
                                                           int t0, int t1, int k, int first, int* pivots, int* m,
                                                           int* qa, int* qb, int* ctl, unsigned long long* keys,
                                                           int* status, unsigned long long* bar) {
    constexpr int VW = W / 4;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    const int sub = gtid % VW, grp = gtid / VW, ngrp = nthreads / VW;
    __shared__ unsigned long long s_red[kSelBlock / kWave];
    unsigned long long epoch = 0;
#define SYNC_OR_LEAVE()                                   \
    if (!sync_grid(bar, epoch)) {                         \
        if (gtid == 0) store_agent(&status[2], 1);       \
        return;                                           \
    }
    for (int t = t0; t < t1; ++t) {
        const int src = (t == 0) ? first : load_agent(&pivots[t]);
        if (gtid == 0) {
            if (t == 0) store_agent(&pivots[0], first);
            atomicMin(&m[src], 0);
            store_agent(&qa[0], src);
            store_agent(&ctl[0], 1);
            store_agent(&ctl[1], 0);
            store_agent(&ctl[2], 0);
        }
        SYNC_OR_LEAVE();
        int level = 0;
        int* cur = qa;
        int* nxt = qb;
        for (;;) {
            const int len = min(load_agent(&ctl[level % 3]), n);
            if (len == 0) break;
            int* tail = &ctl[(level + 1) % 3];
            if (gtid == 0) store_agent(&ctl[(level + 2) % 3], 0);
            const int dv = level + 1;
            const bool pre = len > kSelPrecheck;  // uniform
            for (int base = 0; base < len; base += ngrp) {
                const int qi = base + grp;
                const int v = qi < len ? load_agent(&cur[qi]) : -1;
                int4 nb = make_int4(-1, -1, -1, -1);
                if ((unsigned)v < (unsigned)n) nb = load_agent4(ell + (size_t)v * W + 4 * sub);
                int u[4] = {nb.x, nb.y, nb.z, nb.w};
                int old[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    old[j] = 0;
                    // a stale read of m is never below the current value (m
                    // only falls), so the check never skips a needed atomic
                    if ((unsigned)u[j] < (unsigned)n && (!pre || m[u[j]] > dv)) old[j] = atomicMin(&m[u[j]], dv);
                }
                bool ok[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) ok[j] = (unsigned)u[j] < (unsigned)n && old[j] > dv;
                append4_agent(u, ok, tail, nxt);
                // a row longer than W: its group walks the CSR tail (the
                // continuation mark sits in the group's last lane)
                const bool more = __shfl(nb.w, (lane_id() / VW) * VW + VW - 1) == kEllMore;
                if (__ballot(more) != 0) {  // uniform per wave
                    int e = 0, e1 = 0;
                    if (more) {
                        e = rp[v] + W - 1 + sub;
                        e1 = rp[v + 1];
                    }
                    for (;;) {
                        const bool any = e < e1;
                        if (__ballot(any) == 0) break;
                        int uu[4];
                        int oo[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int ee = e + j * VW;
                            uu[j] = ee < e1 ? ci[ee] : -1;
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            oo[j] = 0;
                            if ((unsigned)uu[j] < (unsigned)n && (!pre || m[uu[j]] > dv))
                                oo[j] = atomicMin(&m[uu[j]], dv);
                        }
                        bool okk[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) okk[j] = (unsigned)uu[j] < (unsigned)n && oo[j] > dv;
                        append4_agent(uu, okk, tail, nxt);
                        e += 4 * VW;
                    }
                }
            }
            SYNC_OR_LEAVE();
            int* tmp = cur;
            cur = nxt;
            nxt = tmp;
            ++level;
        }
        if (t + 1 >= k && t != 0) break;
        // argmax of m: 16-byte agent-scope loads, four in flight
        unsigned long long best = 0;
        const int n4 = n / 4;
        for (int w0 = gtid; w0 < n4; w0 += 4 * nthreads) {
            int4 q[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int w = w0 + j * nthreads;
                q[j] = w < n4 ? load_agent4(m + 4 * (size_t)w) : make_int4(-1, -1, -1, -1);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * (w0 + j * nthreads);
                if (q[j].x >= 0) best = key_max(best, argmax_key(q[j].x, i));
                if (q[j].y >= 0) best = key_max(best, argmax_key(q[j].y, i + 1));
                if (q[j].z >= 0) best = key_max(best, argmax_key(q[j].z, i + 2));
                if (q[j].w >= 0) best = key_max(best, argmax_key(q[j].w, i + 3));
            }
        }
        for (int i = 4 * n4 + gtid; i < n; i += nthreads) best = key_max(best, argmax_key(load_agent(&m[i]), i));
        best = block_max(best, s_red);
        if (threadIdx.x == 0) store_agent(&keys[blockIdx.x], best);
        SYNC_OR_LEAVE();
        if (blockIdx.x == 0 && threadIdx.x < kWave) {  // wave 0 reads the keys, one per lane
            const unsigned long long b = keys_max(keys, (int)gridDim.x);
            if (threadIdx.x == 0) {
                if (t == 0) {
                    if ((int)(b >> 32) == kInf) store_agent(&status[0], 1);
                    store_agent(&status[1], (int)(b >> 32));
                }
                if (t + 1 < k) store_agent(&pivots[t + 1], (int)(0xffffffffu - (unsigned)(b & 0xffffffffu)));
            }
        }
        SYNC_OR_LEAVE();
        if (t == 0 && load_agent(&status[0]) != 0) break;  // disconnected: stop (uniform)
    }
#undef SYNC_OR_LEAVE
}

// Pivots t0 .. t1-1 of max/min sampling in one cooperative launch for
// graphs whose frontiers are narrow: block 0 alone runs each pruned BFS
// (the relaxation of k_select_grid, with workgroup-scope atomics on m, the
// frontier queues in LDS with a global overflow, and four padded rows per
// lane group on levels wider than one pass), so a level costs a workgroup
// barrier instead of a grid barrier; then every block takes part in the
// argmax of m (16-byte loads, four in flight, lowest id on ties).  gq holds
// 3 n ints (frontier overflows, long-row overflow).  status[0] = 1 if the
// first BFS misses a node.
template <int W>
__global__ __launch_bounds__(kBfsBlock) void k_select_hyb(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci, const int* __restrict__ ell,
                                                          int t0, int t1, int k, int first, int* pivots, int* m,
                                                          int* gq, unsigned long long* keys, int* status) {
    cg::grid_group grid = cg::this_grid();
    __shared__ __align__(16) int qpool[2 * kLdsQ + kHeavyCap];
    __shared__ int2 s_slot[3];
    __shared__ unsigned long long s_red[kBfsBlock / kWave];
    int* qa = qpool;
    int* qb = qa + kLdsQ;
    int* lheavy = qb + kLdsQ;
    int* ga = gq;
    int* gb = gq + n;
    int* gh = gb + n;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    for (int t = t0; t < t1; ++t) {
        if (blockIdx.x == 0) {
            const int src = (t == 0) ? first : load_agent(&pivots[t]);
            if (threadIdx.x == 0) {
                if (t == 0) pivots[0] = first;
                m[src] = 0;
                qa[0] = src;
                s_slot[0] = make_int2(0, 0);
            }
            __syncthreads();
            Frontier f{qa, ga, qb, gb, nullptr, lheavy, gh};
            int len = 1;
            for (int level = 0; len > 0; ++level) {
                level_begin(s_slot, level, f);
                const int dv = level + 1;
                len = ell_level_auto<W>(n, rp, ci, ell, len, f, [&](const auto& u, auto& ok) {
                    constexpr int N = sizeof(u) / sizeof(u[0]);
                    int old[N];
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        ok[j] = (unsigned)u[j] < (unsigned)n;  // padding, continuation mark
                        old[j] = ok[j] ? __hip_atomic_fetch_min(&m[u[j]], dv, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_WORKGROUP)
                                       : 0;
                    }
#pragma unroll
                    for (int j = 0; j < N; ++j) ok[j] = ok[j] && old[j] > dv;
                });
                const int* tl = f.lcur;
                f.lcur = f.lnxt;
                f.lnxt = (int*)tl;
                const int* tg = f.gcur;
                f.gcur = f.gnxt;
                f.gnxt = (int*)tg;
            }
        }
        grid_barrier(grid);  // block 0's m is visible to every block
        if (t + 1 >= k && t != 0) break;
        unsigned long long best = 0;
        const int n4 = n / 4;
        const int4* m4 = (const int4*)m;
        for (int w0 = gtid; w0 < n4; w0 += 4 * nthreads) {
            int4 q[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int w = w0 + j * nthreads;
                q[j] = w < n4 ? m4[w] : make_int4(-1, -1, -1, -1);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * (w0 + j * nthreads);
                if (q[j].x >= 0) best = key_max(best, argmax_key(q[j].x, i));
                if (q[j].y >= 0) best = key_max(best, argmax_key(q[j].y, i + 1));
                if (q[j].z >= 0) best = key_max(best, argmax_key(q[j].z, i + 2));
                if (q[j].w >= 0) best = key_max(best, argmax_key(q[j].w, i + 3));
            }
        }
        for (int i = 4 * n4 + gtid; i < n; i += nthreads) best = key_max(best, argmax_key(m[i], i));
        best = block_max(best, s_red);
        if (threadIdx.x == 0) keys[blockIdx.x] = best;
        grid_barrier(grid);
        if (blockIdx.x == 0 && threadIdx.x < kWave) {  // wave 0 reads the keys, one per lane
            const unsigned long long b = keys_max(keys, (int)gridDim.x);
            if (threadIdx.x == 0) {
                if (t == 0) {
                    if ((int)(b >> 32) == kInf) status[0] = 1;
                    status[1] = (int)(b >> 32);
                }
                if (t + 1 < k) pivots[t + 1] = (int)(0xffffffffu - (unsigned)(b & 0xffffffffu));
            }
        }
        grid_barrier(grid);
        if (t == 0 && load_agent(&status[0]) != 0) break;  // disconnected: stop (uniform)
    }
}

// All k pivots in one workgroup (no grid barrier): the same pruned BFS and
// argmax as k_select_all, with the frontier in LDS (global overflow), LDS
// counters and workgroup-scope atomics on m.
template <int VW, bool ROWQ, int PRE>
__global__ __launch_bounds__(kBfsBlock) void k_select_wg(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, int k, int first,
                                                         int* pivots, int* m, int2* queues, int* status) {
    __shared__ int2 sqa[kQcap], sqb[kQcap];
    __shared__ int s_tail, s_len, s_src;
    __shared__ unsigned long long s_red[kBfsBlock / kWave];
    const int sub = threadIdx.x % VW, grp = threadIdx.x / VW, ngrp = blockDim.x / VW;
    int2* ga = queues;
    int2* gb = queues + n;
    if (threadIdx.x == 0) s_src = first;
    __syncthreads();
    for (int t = 0; t < k; ++t) {
        const int src = s_src;
        if (threadIdx.x == 0) {
            pivots[t] = src;
            __hip_atomic_store(&m[src], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            sqa[0] = make_entry<ROWQ>(src, rp);
            s_len = 1;
            s_tail = 0;
        }
        __syncthreads();
        int2* lcur = sqa;
        int2* lnxt = sqb;
        int2* gcur = ga;
        int2* gnxt = gb;
        int level = 0;
        for (;;) {
            const int len = min(s_len, n);
            if (len == 0) break;
            const int dv = level + 1;
            for (int base = 0; base < len; base += ngrp) {
                int qi = base + grp;
                int2 row = make_int2(0, 0);
                if (qi < len) row = entry_row<ROWQ>(queue_get(lcur, gcur, qi), rp, n);
                for (int e = row.x + sub; e < row.y; e += VW) {
                    int v = ci[e];
                    bool push = false;
                    int2 vrow;
                    if ((unsigned)v < (unsigned)n) {
                        // precheck (m only decreases, so a stale value is only larger)
                        const bool try_it = PRE == 0 ? true : PRE == 1 ? m[v] > dv : wg_load(&m[v]) > dv;
                        if (try_it)
                            push = __hip_atomic_fetch_min(&m[v], dv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > dv;
                        if (push) vrow = make_entry<ROWQ>(v, rp);
                    }
                    int slot = wave_append(push, &s_tail);
                    if (push) queue_put(lnxt, gnxt, slot, vrow);
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                s_len = s_tail;
                s_tail = 0;
            }
            int2* t0 = lcur;
            lcur = lnxt;
            lnxt = t0;
            int2* t1 = gcur;
            gcur = gnxt;
            gnxt = t1;
            ++level;
            __syncthreads();
        }
        if (t + 1 >= k && t != 0) break;
        unsigned long long best = 0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            unsigned long long key = ((unsigned long long)(unsigned)wg_load(&m[i]) << 32) |
                                     (unsigned long long)(0xffffffffu - (unsigned)i);
            best = key > best ? key : best;
        }
        best = block_max(best, s_red);
        if (threadIdx.x == 0) {
            if (t == 0 && (int)(best >> 32) == kInf) status[0] = 1;
            s_src = (int)(0xffffffffu - (unsigned)(best & 0xffffffffu));
        }
        __syncthreads();
        if (t == 0 && (int)(best >> 32) == kInf) break;  // disconnected (uniform)
    }
}

// ----------------------------------- one-workgroup selection, LDS-resident

// LDS pool of k_select_ell: the frontier queues, the long-row list and
// either (M8) one state byte per node or (otherwise) one visited bit per
// node.  The state byte holds min(m, kM7Sat) in bits 0-6 and the visited
// flag of the running BFS in bit 7.
constexpr int kSelPool = 155648;
constexpr int kM7Sat = 127;

static bool sel_bits_fit(int n) { return kLdsFixed + lds_bits_bytes(n) <= (size_t)kSelPool; }
static bool sel_m8_fits(int n) { return kLdsFixed + (((size_t)n + 15) & ~(size_t)15) <= (size_t)kSelPool; }


// This thread's best key over m[0..n) (16-byte loads, 4 in flight).  Each
// thread visits its indices in increasing order, so a strict comparison
// keeps the lowest id among equal values.
__device__ __forceinline__ unsigned long long argmax_m_global(const int* __restrict__ m, int n) {
    constexpr int U = 4;
    const int n4 = n / 4;
    const int4* m4 = (const int4*)m;
    int bv = -1, bi = 0;
    for (int w0 = threadIdx.x; w0 < n4; w0 += U * blockDim.x) {
        int4 q[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int w = w0 + j * (int)blockDim.x;
            q[j] = w < n4 ? m4[w] : make_int4(-1, -1, -1, -1);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int i = 4 * (w0 + j * (int)blockDim.x);
            if (q[j].x > bv) { bv = q[j].x; bi = i; }
            if (q[j].y > bv) { bv = q[j].y; bi = i + 1; }
            if (q[j].z > bv) { bv = q[j].z; bi = i + 2; }
            if (q[j].w > bv) { bv = q[j].w; bi = i + 3; }
        }
    }
    unsigned long long best = bv >= 0 ? argmax_key(bv, bi) : 0ull;
    for (int i = 4 * n4 + threadIdx.x; i < n; i += blockDim.x) {  // tail
        const unsigned long long key = argmax_key(m[i], i);
        if (key > best) best = key;
    }
    return best;
}

// Exact argmax when the state bytes saturate: a byte below kM7Sat is the
// value, a saturated byte defers to global m (which holds every value of 127
// and above; it is not kept current below).
__device__ __forceinline__ unsigned long long argmax_m7_global(const unsigned char* m8, const int* __restrict__ m,
                                                               int n) {
    unsigned long long best = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int b = m8[i] & 0x7f;
        const int v = b < kM7Sat ? b : m[i];
        const unsigned long long key = argmax_key(v, i);
        if (key > best) best = key;
    }
    return best;
}

// Same over the LDS state bytes (16 bytes per read): the value is bits 0-6;
// the pass also clears the visited flags (bit 7) for the next BFS.  The
// bytes are 16-byte aligned and padded with zeros to a multiple of 16.
__device__ __forceinline__ unsigned long long argmax_m7_clear(unsigned char* m8, int n) {
    uint4* w16 = (uint4*)m8;
    const int nw = (n + 15) / 16;
    int bv = -1, bi = 0;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) {
        uint4 q = w16[w];
        q.x &= 0x7f7f7f7fu;
        q.y &= 0x7f7f7f7fu;
        q.z &= 0x7f7f7f7fu;
        q.w &= 0x7f7f7f7fu;
        w16[w] = q;
        const unsigned part[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int val = (int)((part[a] >> (8 * b)) & 127u);
                if (val > bv) {
                    bv = val;
                    bi = 16 * w + 4 * a + b;
                }
            }
        }
    }
    return bv >= 0 ? argmax_key(bv, bi) : 0ull;
}

// Frontier nodes that one pass of wave 0 covers in wave_levels (W / 4
// lanes per node, as in the block levels).
template <int W>
constexpr int wave_level_nodes() {
    return kWave / (W / 4);
}

// Levels whose frontier one wave covers in one pass, run in wave 0 alone
// (state bytes): W / 4 lanes per frontier node take four ELL slots each, the
// whole wave then takes the CSR tails of long rows, 64 arcs at a time; the
// claims are the block levels' and the wave ranks its appends with ballots,
// so neither an LDS counter nor a barrier separates these levels (LDS
// operations of one wave complete in order).  Runs while the frontier holds
// 1 .. wave_level_nodes<W>() nodes and the next level stays below kM7Sat
// (where the state byte alone decides); returns the frontier size, advances
// level and counts the queue swaps.
template <int W, int P>
__device__ __forceinline__ int wave_levels(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                           const int* __restrict__ ell, unsigned char* m8, const Frontier& f0,
                                           int len, int& level, int& swaps) {
    constexpr int G = W / 4;
    const int lane = lane_id(), sub = lane % G;
    const int* lcur = f0.lcur;
    int* lnxt = f0.lnxt;
    int* gnxt = f0.gnxt;
    const int* gcur = f0.gcur;
    while (len > 0 && len <= P * wave_level_nodes<W>() && level + 1 < kM7Sat) {
        const int dv = level + 1;
        int v[P];
        int4 nb[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int q = p * wave_level_nodes<W>() + lane / G;
            v[p] = q < len ? lcur[q] : -1;  // the LDS part holds the frontier
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            nb[p] = make_int4(-1, -1, -1, -1);
            if ((unsigned)v[p] < (unsigned)n) nb[p] = *(const int4*)(ell + (size_t)v[p] * W + 4 * sub);
        }
        int cnt = 0;
        // claim u and append it if it joins the next frontier (uniform call)
        auto take = [&](int u, unsigned old) {
            const unsigned ob = (old >> (8 * (u & 3))) & 0xffu;
            const bool ok = (unsigned)u < (unsigned)n && !(ob & 0x80u) && (int)(ob & 0x7fu) > dv;
            if (ok) m8[u] = (unsigned char)(0x80 | dv);
            const uint64_t mk = __ballot(ok);
            if (ok) {
                const int slot = cnt + mask_rank(mk);
                if (slot < kLdsQ)
                    lnxt[slot] = u;
                else
                    gnxt[slot - kLdsQ] = u;
            }
            cnt += __popcll(mk);
        };
        auto claim = [&](int u) {
            return (unsigned)u < (unsigned)n ? atomicOr((unsigned*)(m8 + (u & ~3)), 0x80u << (8 * (u & 3)))
                                             : 0x80808080u;
        };
        unsigned old[4 * P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            old[4 * p] = claim(nb[p].x);
            old[4 * p + 1] = claim(nb[p].y);
            old[4 * p + 2] = claim(nb[p].z);
            old[4 * p + 3] = claim(nb[p].w);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            take(nb[p].x, old[4 * p]);
            take(nb[p].y, old[4 * p + 1]);
            take(nb[p].z, old[4 * p + 2]);
            take(nb[p].w, old[4 * p + 3]);
        }
        // long rows: the whole wave over each tail, 64 arcs at a time
#pragma unroll
        for (int p = 0; p < P; ++p) {
          uint64_t hm = __ballot(sub == G - 1 && nb[p].w == kEllMore);
          while (hm) {
            const int src_lane = __builtin_ctzll(hm);
            hm &= hm - 1;
            const int h = __shfl(v[p], src_lane);
            const int e1 = rp[h + 1];
            for (int e = rp[h] + W - 1 + lane; __any(e < e1); e += kWave) {
                const int t = e < e1 ? ci[e] : -1;
                take(t, claim(t));
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
        len = cnt;
        const int* tl = lcur;
        lcur = lnxt;
        lnxt = (int*)tl;
        const int* tg = gcur;
        gcur = gnxt;
        gnxt = (int*)tg;
        ++swaps;
        ++level;
    }
    return len;
}

// All k pivots in one workgroup: for each new pivot the BFS that only
// continues through nodes whose distance to it is below m (as k_select_all),
// on LDS-resident levels.
//   M8: one LDS state byte per node.  A claim is one LDS atomic OR that sets
//       the node's visited flag and returns its old byte, i.e. the flag and
//       min(m, 127) together; below 127 the pruning test m > dv is exact on
//       the byte, at or above it global m decides.  The argmax scans the
//       bytes (and clears the flags) unless the maximum is saturated.
//   otherwise: LDS visited bits, global m.
// The claiming lane owns m[v] for the level and writes it with plain
// stores.  gq holds 3 n ints.
template <int W, bool M8, int SPOOL = kSelPool>
__device__ __forceinline__ void select_ell_body(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const int* __restrict__ ell, int k, int first, int* pivots, int* m,
                                                int* gq, int* status, int wave_mode = 1) {
    __shared__ __align__(16) unsigned char pool[SPOOL];
    __shared__ int2 s_slot[3];
    __shared__ int s_src;
    __shared__ int s_wave[3];
    __shared__ unsigned long long s_red[kBfsBlock / kWave];
    int* qa = (int*)pool;
    int* qb = qa + kLdsQ;
    int* lheavy = qb + kLdsQ;
    unsigned* bits = (unsigned*)(lheavy + kHeavyCap);  // !M8: visited bits
    unsigned char* m8 = (unsigned char*)bits;          // M8: state bytes (16-byte aligned)
    const int nbw = (n + 31) / 32;
    int* ga = gq;
    int* gb = gq + n;
    int* gh = gb + n;

    if (M8)
        for (int i = threadIdx.x; i < ((n + 15) & ~15); i += blockDim.x) m8[i] = i < n ? (unsigned char)kM7Sat : 0;
    if (threadIdx.x == 0) s_src = first;
    __syncthreads();
    for (int t = 0; t < k; ++t) {
        const int src = s_src;
        if (!M8)
            for (int w = threadIdx.x; w < nbw; w += blockDim.x) bits[w] = 0u;
        __syncthreads();
        if (threadIdx.x == 0) {
            pivots[t] = src;
            m[src] = 0;
            if (M8)
                m8[src] = 0x80;  // m = 0, visited
            else
                bits[src >> 5] |= 1u << (src & 31);
            qa[0] = src;
            s_slot[0] = make_int2(0, 0);
        }
        __syncthreads();
        Frontier f{qa, ga, qb, gb, nullptr, lheavy, gh};
        int len = 1;
        for (int level = 0; len > 0; ++level) {
            if (M8 && wave_mode > 0 && len <= wave_mode * wave_level_nodes<W>() && level + 1 < kM7Sat) {  // uniform
                if (threadIdx.x < kWave) {
                    int lv = level, sw = 0;
                    const int nl = wave_mode == 1 ? wave_levels<W, 1>(n, rp, ci, ell, m8, f, len, lv, sw)
                                                  : wave_levels<W, 2>(n, rp, ci, ell, m8, f, len, lv, sw);
                    if (threadIdx.x == 0) {
                        s_wave[0] = nl;
                        s_wave[1] = lv;
                        s_wave[2] = sw;
                        // the block levels' counters: clear for whichever level comes next
                        s_slot[0] = s_slot[1] = s_slot[2] = make_int2(0, 0);
                    }
                }
                __syncthreads();
                len = s_wave[0];
                const int nlev = s_wave[1], sw = s_wave[2];
                if (sw & 1) {
                    const int* tl = f.lcur;
                    f.lcur = f.lnxt;
                    f.lnxt = (int*)tl;
                    const int* tg = f.gcur;
                    f.gcur = f.gnxt;
                    f.gnxt = (int*)tg;
                }
                level = nlev - 1;  // the loop steps to nlev
                continue;
            }
            level_begin(s_slot, level, f);
            const int dv = level + 1;
            len = ell_level_auto<W>(n, rp, ci, ell, len, f, [&](const auto& u, auto& ok) {
                constexpr int N = sizeof(u) / sizeof(u[0]);
                int mv[N];
                if (M8) {
                    // claim and read the old state byte with one atomic per node
                    unsigned old[N];
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        ok[j] = (unsigned)u[j] < (unsigned)n;  // padding, continuation mark, bad index
                        const int sh = 8 * (u[j] & 3);
                        old[j] = ok[j] ? atomicOr((unsigned*)(m8 + (u[j] & ~3)), 0x80u << sh) : 0x80u;
                    }
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        const unsigned ob = (old[j] >> (8 * (u[j] & 3))) & 0xffu;
                        ok[j] = ok[j] && !(ob & 0x80u);
                        mv[j] = (int)(ob & 0x7fu);
                    }
                    if (dv >= kM7Sat) {  // uniform: the byte is saturated, global m decides
#pragma unroll
                        for (int j = 0; j < N; ++j)
                            if (ok[j] && mv[j] >= kM7Sat) mv[j] = m[u[j]];
                    }
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        // a saturated byte below level 127 means m >= 127 > dv
                        ok[j] = ok[j] && (mv[j] > dv || (mv[j] >= kM7Sat && dv < kM7Sat));
                        if (ok[j]) m8[u[j]] = (unsigned char)(0x80 | min(dv, kM7Sat));
                    }
                    // global m only holds the values the byte cannot (>= 127):
                    // no global store on the levels below 127
                    if (dv >= kM7Sat) {  // uniform
#pragma unroll
                        for (int j = 0; j < N; ++j)
                            if (ok[j]) m[u[j]] = dv;
                    }
                } else {
                    claim(u, ok, bits, n);
                    // all reads first, then all stores: a wait for a read must
                    // not also wait for this level's stores
#pragma unroll
                    for (int j = 0; j < N; ++j) mv[j] = ok[j] ? m[u[j]] : 0;
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        ok[j] = ok[j] && mv[j] > dv;
                        if (ok[j]) m[u[j]] = dv;
                    }
                }
            });
            const int* tl = f.lcur;
            f.lcur = f.lnxt;
            f.lnxt = (int*)tl;
            const int* tg = f.gcur;
            f.gcur = f.gnxt;
            f.gnxt = (int*)tg;
        }
        if (t + 1 >= k && t != 0) break;
        unsigned long long best;
        if (M8) {
            best = block_max(argmax_m7_clear(m8, n), s_red);
            if ((int)(best >> 32) >= kM7Sat) best = block_max(argmax_m7_global(m8, m, n), s_red);  // uniform
        } else {
            best = block_max(argmax_m_global(m, n), s_red);
        }
        if (threadIdx.x == 0) {
            if (t == 0 && (int)(best >> 32) == kInf) status[0] = 1;
            s_src = (int)(0xffffffffu - (unsigned)(best & 0xffffffffu));
        }
        __syncthreads();
        if (t == 0 && (int)(best >> 32) == kInf) break;  // disconnected (uniform)
    }
}

template <int W, bool M8>
__global__ __launch_bounds__(kBfsBlock) void k_select_ell(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci, const int* __restrict__ ell,
                                                          int k, int first, int* pivots, int* m, int* gq,
                                                          int* status, int wave_mode) {
    select_ell_body<W, M8>(n, rp, ci, ell, k, first, pivots, m, gq, status, wave_mode);
}

template <int W, bool M8>
static hipError_t launch_select_ell_t(hipStream_t s, int n, const int* rp, const int* ci, const int* ell, int k,
                                      int first, int* pivots, int* m, int* q, int* status) {
    int threads = kBfsBlock;
    const int v = variant("select_threads");  // tuning override: 256, 512 or 1024
    if (v == 256 || v == 512) threads = v;
    // small frontiers in one wave, one pass per level (variant select_wave:
    // -1 = block levels only, 2 = up to two passes)
    const int wv = variant("select_wave", 1);
    const int wave_mode = std::max(0, std::min(2, wv));
    hipLaunchKernelGGL((k_select_ell<W, M8>), dim3(1), dim3(threads), 0, s, n, rp, ci, ell, k, first, pivots, m,
                       q, status, wave_mode);
    return hipGetLastError();
}

static hipError_t launch_select_ell(int W, bool m8, hipStream_t s, int n, const int* rp, const int* ci,
                                    const int* ell, int k, int first, int* pivots, int* m, int* q, int* status) {
    if (m8) {
        if (W == 8) return launch_select_ell_t<8, true>(s, n, rp, ci, ell, k, first, pivots, m, q, status);
        if (W == 16) return launch_select_ell_t<16, true>(s, n, rp, ci, ell, k, first, pivots, m, q, status);
        return launch_select_ell_t<32, true>(s, n, rp, ci, ell, k, first, pivots, m, q, status);
    }
    if (W == 8) return launch_select_ell_t<8, false>(s, n, rp, ci, ell, k, first, pivots, m, q, status);
    if (W == 16) return launch_select_ell_t<16, false>(s, n, rp, ci, ell, k, first, pivots, m, q, status);
    return launch_select_ell_t<32, false>(s, n, rp, ci, ell, k, first, pivots, m, q, status);
}

template <int VW, bool ROWQ, int PRE>
static void launch_select_wg_t(hipStream_t s, int n, const int* rp, const int* ci, int k, int first, int* pivots,
                               int* m, int2* q, int* status) {
    hipLaunchKernelGGL((k_select_wg<VW, ROWQ, PRE>), dim3(1), dim3(kBfsBlock), 0, s, n, rp, ci, k, first, pivots, m, q,
                       status);
}

template <int VW>
static void launch_select_wg_v(hipStream_t s, int n, const int* rp, const int* ci, int k, int first, int* pivots,
                               int* m, int2* q, int* status) {
    // queue style and relaxation precheck: defaults measured on MI355X; the
    // environment overrides them for tuning
    const int rowq = variant("select_rowq"), pre = variant("select_pre");
    if (rowq != 2) {  // row bounds in the queue (2 = node ids; tuning)
        if (pre == 1) launch_select_wg_t<VW, true, 1>(s, n, rp, ci, k, first, pivots, m, q, status);
        else if (pre == 3) launch_select_wg_t<VW, true, 0>(s, n, rp, ci, k, first, pivots, m, q, status);
        else launch_select_wg_t<VW, true, 2>(s, n, rp, ci, k, first, pivots, m, q, status);
    } else {
        if (pre == 2) launch_select_wg_t<VW, false, 2>(s, n, rp, ci, k, first, pivots, m, q, status);
        else if (pre == 3) launch_select_wg_t<VW, false, 0>(s, n, rp, ci, k, first, pivots, m, q, status);
        else launch_select_wg_t<VW, false, 1>(s, n, rp, ci, k, first, pivots, m, q, status);
    }
}

static hipError_t launch_select_wg(int vw, hipStream_t s, int n, const int* rp, const int* ci, int k, int first,
                                   int* pivots, int* m, int2* q, int* status) {
    switch (vw) {
        case 2: launch_select_wg_v<2>(s, n, rp, ci, k, first, pivots, m, q, status); break;
        case 4: launch_select_wg_v<4>(s, n, rp, ci, k, first, pivots, m, q, status); break;
        case 8: launch_select_wg_v<8>(s, n, rp, ci, k, first, pivots, m, q, status); break;
        case 16: launch_select_wg_v<16>(s, n, rp, ci, k, first, pivots, m, q, status); break;
        case 32: launch_select_wg_v<32>(s, n, rp, ci, k, first, pivots, m, q, status); break;
        default: launch_select_wg_v<64>(s, n, rp, ci, k, first, pivots, m, q, status); break;
    }
    return hipGetLastError();
}

template <int VW>
static hipError_t launch_select_all(int blocks, hipStream_t s, int n, const int* rp, const int* ci, int k,
                                    int first, int* pivots, int* m, int* qa, int* qb, int* ctl,
                                    unsigned long long* keys, int* status) {
    void* args[] = {&n, &rp, &ci, &k, &first, &pivots, &m, &qa, &qb, &ctl, &keys, &status};
    return hipLaunchCooperativeKernel((const void*)k_select_all<VW>, dim3(blocks), dim3(kSelBlock), args, 0, s);
}


template <int VW>
static hipError_t launch_select(int blocks, hipStream_t s, int n, const int* rp, const int* ci,
                                int t, int k, int first, int* pivots, int* m, int* vis, int* qa,
                                int* qb, int* ctl, unsigned long long* keys, int* status) {
    void* args[] = {&n, &rp, &ci, &t, &k, &first, &pivots, &m, &vis, &qa, &qb, &ctl, &keys, &status};
    return hipLaunchCooperativeKernel((const void*)k_select<VW>, dim3(blocks), dim3(kSelBlock), args,
                                      0, s);
}

template <int W>
static hipError_t launch_select_grid_w(int blocks, hipStream_t s, int n, const int* rp, const int* ci, const int* ell,
                                       int t0, int t1, int k, int first, int* pivots, int* m, int* qa, int* qb,
                                       int* ctl, unsigned long long* keys, int* status, unsigned long long* bar) {
    void* args[] = {&n, &rp, &ci, &ell, &t0, &t1, &k, &first, &pivots, &m, &qa, &qb, &ctl, &keys, &status, &bar};
    return hipLaunchCooperativeKernel((const void*)k_select_grid<W>, dim3(blocks), dim3(kSelBlock), args, 0, s);
}

// bar: a zeroed 64-bit barrier counter for this launch alone
static hipError_t launch_select_grid(int W, int blocks, hipStream_t s, int n, const int* rp, const int* ci,
                                     const int* ell, int t0, int t1, int k, int first, int* pivots, int* m, int* qa,
                                     int* qb, int* ctl, unsigned long long* keys, int* status,
                                     unsigned long long* bar) {
    if (W == 8)
        return launch_select_grid_w<8>(blocks, s, n, rp, ci, ell, t0, t1, k, first, pivots, m, qa, qb, ctl, keys,
                                       status, bar);
    if (W == 16)
        return launch_select_grid_w<16>(blocks, s, n, rp, ci, ell, t0, t1, k, first, pivots, m, qa, qb, ctl, keys,
                                        status, bar);
    return launch_select_grid_w<32>(blocks, s, n, rp, ci, ell, t0, t1, k, first, pivots, m, qa, qb, ctl, keys,
                                    status, bar);
}

template <int W>
static hipError_t launch_select_hyb_w(int blocks, hipStream_t s, int n, const int* rp, const int* ci, const int* ell,
                                      int t0, int t1, int k, int first, int* pivots, int* m, int* gq,
                                      unsigned long long* keys, int* status) {
    void* args[] = {&n, &rp, &ci, &ell, &t0, &t1, &k, &first, &pivots, &m, &gq, &keys, &status};
    return hipLaunchCooperativeKernel((const void*)k_select_hyb<W>, dim3(blocks), dim3(kBfsBlock), args, 0, s);
}

static hipError_t launch_select_hyb(int W, int blocks, hipStream_t s, int n, const int* rp, const int* ci,
                                    const int* ell, int t0, int t1, int k, int first, int* pivots, int* m, int* gq,
                                    unsigned long long* keys, int* status) {
    if (W == 8)
        return launch_select_hyb_w<8>(blocks, s, n, rp, ci, ell, t0, t1, k, first, pivots, m, gq, keys, status);
    if (W == 16)
        return launch_select_hyb_w<16>(blocks, s, n, rp, ci, ell, t0, t1, k, first, pivots, m, gq, keys, status);
    return launch_select_hyb_w<32>(blocks, s, n, rp, ci, ell, t0, t1, k, first, pivots, m, gq, keys, status);
}

static int select_hyb_max_blocks(int W) {
    int a = 0;
    const void* f = W == 8 ? (const void*)k_select_hyb<8> : W == 16 ? (const void*)k_select_hyb<16>
                                                                     : (const void*)k_select_hyb<32>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, f, kBfsBlock, 0) != hipSuccess) a = 1;
    return std::max(1, a) * num_cus();
}

static int select_grid_max_blocks(int W) {
    int a = 0;
    const void* f = W == 8 ? (const void*)k_select_grid<8> : W == 16 ? (const void*)k_select_grid<16>
                                                                       : (const void*)k_select_grid<32>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, f, kSelBlock, 0) != hipSuccess) a = 1;
    return std::max(1, a) * num_cus();
}

template <int VW>
static int select_max_blocks() {
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void*)k_select<VW>, kSelBlock, 0) != hipSuccess)
        a = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)k_select_all<VW>, kSelBlock, 0) !=
        hipSuccess)
        b = 1;
    return std::max(1, std::min(a, b)) * num_cus();
}

// One workgroup up to this many nodes (its levels cost no grid barrier); the
// cooperative grid above (frontiers too wide for one workgroup).
constexpr long long kSelOneWgMaxN = 1LL << 18;
constexpr int kSelGridBlocks = 32;
constexpr int kSelHybBlocks = 64;  // grid of the hybrid form (its blocks only share the argmax)

ssm_status select_pivots(const ssm_csr* g, int32_t k, int32_t first, int32_t* pivots, hipStream_t s) {
    const int n = g->n;
    // workspace: m[n], vis[n], qa[n], qb[n], ctl[4], status[3], barrier counters, keys[max blocks]
    int vw = virtual_warp(g);
    int maxb = 1;
    switch (vw) {
        case 2: maxb = select_max_blocks<2>(); break;
        case 4: maxb = select_max_blocks<4>(); break;
        case 8: maxb = select_max_blocks<8>(); break;
        case 16: maxb = select_max_blocks<16>(); break;
        case 32: maxb = select_max_blocks<32>(); break;
        default: maxb = select_max_blocks<64>(); break;
    }
    // Grid size for the cooperative forms: a grid barrier per BFS level costs
    // more with more blocks, so a few dozen (measured best on MI355X for
    // 1M-node power-law and 3M-node mesh graphs).
    int blocks = std::max(1, std::min(std::min(maxb, kSelGridBlocks), div_up(n, 8192)));
    if (variant("select_blocks") > 0) blocks = std::min(maxb, variant("select_blocks"));
    // m[n], vis[n], queue area (4n ints: two int queues of n, or two int2
    // queues of n for the one-workgroup kernel), control words, and two
    // 64-bit grid barrier counters on lines of their own
    size_t ints = 6 * (size_t)n + 128;
    int* ws = nullptr;
    unsigned long long* keys = nullptr;
    ssm_status st = salloc((void**)&ws, sizeof(int) * ints);
    if (st != SSM_OK) return st;
    constexpr int kKeysMax = 4096;  // partial argmax keys: room for any grid below
    st = salloc((void**)&keys, sizeof(unsigned long long) * std::max(blocks, kKeysMax));
    if (st != SSM_OK) {
        sfree(ws);
        return st;
    }
    int* m = ws;
    int* vis = ws + n;
    int* qa = ws + 2 * (size_t)n;
    int* qb = ws + 3 * (size_t)n;
    int* ctl = ws + 6 * (size_t)n;
    int* status = ctl + 4;
    unsigned long long* bars = (unsigned long long*)(ctl + 32);  // bars[0], bars[16]: one per launch
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3(std::min(div_up(n, 256), 4096)), dim3(256), 0, s, m, kInf, (long long)n);
    hipLaunchKernelGGL(k_fill_int, dim3(std::min(div_up(n, 256), 4096)), dim3(256), 0, s, vis, -1, (long long)n);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(128), 0, s, ctl, 0, (long long)128);
    hipLaunchKernelGGL(k_fill_int, dim3(std::min(div_up(4 * (long long)n, 256), 4096)), dim3(256), 0, s, qa, 0,
                       4 * (long long)n);
    e = hipGetLastError();
    // Mode: one workgroup (no grid barrier) unless the frontiers are large.
    // 1 = one workgroup, 2 = cooperative grid over CSR rows, 3 = per pivot,
    // 4 = cooperative grid over padded rows
    int mode = variant("select_mode");
    if (mode < 1 || mode > 4) mode = (long long)n <= kSelOneWgMaxN ? 1 : 4;
    const bool per_pivot = mode == 3;
    // One workgroup: the LDS-resident form when the visited bits fit (tuning
    // override SSM_SELECT_ELL=2 keeps the global-memory form).
    int* ell = nullptr;
    const bool use_ell = mode == 1 && sel_bits_fit(n) && variant("select_ell") != 2;
    const int W = ell_width(g);
    if (use_ell && e == hipSuccess) {
        st = salloc((void**)&ell, sizeof(int) * (size_t)n * W);
        if (st != SSM_OK) {
            (void)hipStreamSynchronize(s);  // fills queued on ws: idle before reuse
            sfree(ws);
            sfree(keys);
            return st;
        }
        e = ell_build(g, W, ell, s);
        // with the byte copy of m when it fits (tuning override SSM_SELECT_M8=2: without)
        const bool m8 = sel_m8_fits(n) && variant("select_m8") != 2;
        if (e == hipSuccess)
            e = launch_select_ell(W, m8, s, n, g->row_ptr, g->col_idx, ell, k, first, pivots, m, qa, status);
    } else if (mode == 1 && e == hipSuccess) {
        e = launch_select_wg(vw, s, n, g->row_ptr, g->col_idx, k, first, pivots, m, (int2*)qa, status);
    }
    if (mode == 2 && e == hipSuccess) {
        switch (vw) {
            case 2: e = launch_select_all<2>(blocks, s, n, g->row_ptr, g->col_idx, k, first, pivots, m, qa, qb, ctl, keys, status); break;
            case 4: e = launch_select_all<4>(blocks, s, n, g->row_ptr, g->col_idx, k, first, pivots, m, qa, qb, ctl, keys, status); break;
            case 8: e = launch_select_all<8>(blocks, s, n, g->row_ptr, g->col_idx, k, first, pivots, m, qa, qb, ctl, keys, status); break;
            case 16: e = launch_select_all<16>(blocks, s, n, g->row_ptr, g->col_idx, k, first, pivots, m, qa, qb, ctl, keys, status); break;
            case 32: e = launch_select_all<32>(blocks, s, n, g->row_ptr, g->col_idx, k, first, pivots, m, qa, qb, ctl, keys, status); break;
            default: e = launch_select_all<64>(blocks, s, n, g->row_ptr, g->col_idx, k, first, pivots, m, qa, qb, ctl, keys, status); break;
        }
    }
    if (mode == 4 && e == hipSuccess) {
        // pivot 0's BFS on the default grid, then a grid sized by the graph's
        // mean frontier, n / (eccentricity of pivot 0 + 1): a level costs a
        // grid barrier whose time grows with the blocks, so narrow frontiers
        // (long paths, meshes) take fewer blocks (measured on MI355X: a
        // 3.25M-node mesh is fastest at 16, a 1M-node power-law graph at 32)
        const int W = ell_width(g);
        const int gmax = std::min(select_grid_max_blocks(W), kKeysMax);
        int b0 = std::max(1, std::min(std::min(gmax, kSelGridBlocks), div_up(n, 8192)));
        st = salloc((void**)&ell, sizeof(int) * (size_t)n * W);
        if (st != SSM_OK) {
            (void)hipStreamSynchronize(s);
            sfree(ws);
            sfree(keys);
            return st;
        }
        e = ell_build(g, W, ell, s);
        if (e == hipSuccess)
            e = launch_select_grid(W, b0, s, n, g->row_ptr, g->col_idx, ell, 0, 1, k, first, pivots, m, qa, qb, ctl,
                                   keys, status, bars);
        int hs[3] = {0, 0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(hs, status, sizeof hs, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess && hs[0] == 0 && hs[2] == 0 && k > 1) {
            const double mean_front = (double)n / ((double)hs[1] + 1.0);
            // variant select_hyb = 1: block 0 runs each pruned BFS alone and
            // the grid joins for the argmax (measured on MI355X: 216 against
            // 170 ms on a 3.25M-node mesh, where one CU still pays the same
            // chain of dependent memory round trips per level)
            const bool hyb = variant("select_hyb") == 1;
            if (hyb) {
                int* gq = nullptr;
                st = salloc((void**)&gq, sizeof(int) * 3 * (size_t)n);
                if (st == SSM_OK) {
                    int bh = std::max(1, std::min({select_hyb_max_blocks(W), kKeysMax, kSelHybBlocks}));
                    if (variant("select_blocks") > 0) bh = std::max(1, std::min(bh, variant("select_blocks")));
                    e = launch_select_hyb(W, bh, s, n, g->row_ptr, g->col_idx, ell, 1, k, k, first, pivots, m, gq,
                                          keys, status);
                    (void)hipStreamSynchronize(s);  // idle before the scratch is reused
                    sfree(gq);
                } else {
                    (void)hipStreamSynchronize(s);
                    sfree(ws);
                    sfree(keys);
                    sfree(ell);
                    return st;
                }
            } else {
                int b1 = mean_front < 4096.0 ? std::min(b0, kSelGridBlocks / 2) : b0;
                if (variant("select_blocks") > 0) b1 = std::min(gmax, variant("select_blocks"));
                b1 = std::max(1, std::min(b1, gmax));
                e = launch_select_grid(W, b1, s, n, g->row_ptr, g->col_idx, ell, 1, k, k, first, pivots, m, qa, qb,
                                       ctl, keys, status, bars + 16);
            }
        }
    }
    for (int t = 0; per_pivot && t < k && e == hipSuccess; ++t) {
        switch (vw) {
            case 2: e = launch_select<2>(blocks, s, n, g->row_ptr, g->col_idx, t, k, first, pivots, m, vis, qa, qb, ctl, keys, status); break;
            case 4: e = launch_select<4>(blocks, s, n, g->row_ptr, g->col_idx, t, k, first, pivots, m, vis, qa, qb, ctl, keys, status); break;
            case 8: e = launch_select<8>(blocks, s, n, g->row_ptr, g->col_idx, t, k, first, pivots, m, vis, qa, qb, ctl, keys, status); break;
            case 16: e = launch_select<16>(blocks, s, n, g->row_ptr, g->col_idx, t, k, first, pivots, m, vis, qa, qb, ctl, keys, status); break;
            case 32: e = launch_select<32>(blocks, s, n, g->row_ptr, g->col_idx, t, k, first, pivots, m, vis, qa, qb, ctl, keys, status); break;
            default: e = launch_select<64>(blocks, s, n, g->row_ptr, g->col_idx, t, k, first, pivots, m, vis, qa, qb, ctl, keys, status); break;
        }
    }
    int hstatus[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hstatus, status, sizeof hstatus, hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused (also after an error)
    sfree(ws);
    sfree(keys);
    if (ell) sfree(ell);
    if (e != hipSuccess) return hip_fail(e, "pivot selection");
    if (hstatus[2]) return fail(SSM_E_DEVICE, "pivot selection: a grid barrier did not fill and was aborted");
    if (hstatus[0]) return fail(SSM_E_DISCONNECTED, "graph is not connected (the first BFS missed nodes)");
    return SSM_OK;
}

// ---------------------------------------------------------------- regions

constexpr int kMaxCand = 4;
constexpr int kRegOneWgMax = 16384;  // tied nodes resolved by one workgroup

// Per node: delta = min_t dist[t][i]; the candidates (ranks at that
// distance, ascending, the first kMaxCand kept; cand.w = count).  A node with
// one candidate joins it at once.  aux[0] = max delta, aux[1] = tied nodes.
__global__ __launch_bounds__(256) void k_reg_scan(int n, int k, const int* __restrict__ dist, int* __restrict__ delta,
                           int* __restrict__ region, int4* __restrict__ cand, int* aux) {
    int tied = 0, dm = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int best = kInf, cnt = 0;
        int c[kMaxCand] = {-1, -1, -1, -1};
        constexpr int U = 8;  // distance loads in flight
        for (int t0 = 0; t0 < k; t0 += U) {
            int dv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) dv[j] = t0 + j < k ? dist[(size_t)(t0 + j) * n + i] : kInf;
#pragma unroll
            for (int j = 0; j < U; ++j) {  // ranks in ascending order
                if (t0 + j >= k) break;
                const int d = dv[j], t = t0 + j;
                if (d < best) {
                    best = d;
                    cnt = 1;
                    c[0] = t;
                } else if (d == best) {
                    if (cnt < kMaxCand) c[cnt] = t;
                    ++cnt;
                }
            }
        }
        delta[i] = best;
        region[i] = cnt == 1 ? c[0] : -1;
        cand[i] = make_int4(c[0], c[1], c[2], cnt);
        tied += cnt > 1;
        dm = best > dm ? best : dm;
    }
    __shared__ int red[256 / kWave];
    tied = block_sum(tied, red);
    dm = block_max(dm, red);
    if (threadIdx.x == 0) {  // one atomic per block
        if (tied) atomicAdd(&aux[1], tied);
        atomicMax(&aux[0], dm);
    }
}

constexpr int kRegHistLds = 8192;  // counters a block keeps in LDS before flushing

// Histogram of single-candidate nodes per (pivot, level) and count of tied
// nodes per level.  With LDS the block counts into LDS ((k + 1) L counters)
// and adds its nonzero counts to the global ones at the end.
template <bool LDS>
__global__ __launch_bounds__(256) void k_reg_hist(int n, int k, int L, const int* __restrict__ delta,
                                                  const int4* __restrict__ cand, int* __restrict__ U,
                                                  int* __restrict__ tcount) {
    extern __shared__ int sh[];
    int* sU = sh;                   // [k][L]
    int* sT = sh + (size_t)k * L;   // [L]
    if (LDS) {
        for (int q = threadIdx.x; q < (k + 1) * L; q += blockDim.x) sh[q] = 0;
        __syncthreads();
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int4 c = cand[i];
        const int l = delta[i];
        if (c.w == 1)
            atomicAdd(LDS ? &sU[(size_t)c.x * L + l] : &U[(size_t)c.x * L + l], 1);
        else
            atomicAdd(LDS ? &sT[l] : &tcount[l], 1);
    }
    if (LDS) {
        __syncthreads();
        for (int q = threadIdx.x; q < (k + 1) * L; q += blockDim.x) {
            const int v = sh[q];
            if (v) atomicAdd(q < k * L ? &U[q] : &tcount[q - k * L], v);
        }
    }
}

// Exclusive prefix over levels (one thread; L is small).
__global__ void k_reg_prefix(int L, const int* __restrict__ tcount, int* __restrict__ tstart,
                             int* __restrict__ cursor) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int acc = 0;
        for (int l = 0; l < L; ++l) {
            tstart[l] = acc;
            cursor[l] = acc;
            acc += tcount[l];
        }
        tstart[L] = acc;
    }
}

// Lists the tied nodes by level with one global atomic per node (many levels).
__global__ void k_reg_scatter_global(int n, const int* __restrict__ delta, const int4* __restrict__ cand,
                                     int* __restrict__ cursor, int* __restrict__ list) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (cand[i].w > 1) list[atomicAdd(&cursor[delta[i]], 1)] = i;
}

// Lists the tied nodes by level: a block counts its tied nodes per level in
// LDS, reserves one range per level with a global atomic, then places them
// (the order inside a level does not matter to the resolution).  LDS holds
// 2 L ints.
__global__ __launch_bounds__(256) void k_reg_scatter(int n, int L, const int* __restrict__ delta,
                                                     const int4* __restrict__ cand, int* __restrict__ cursor,
                                                     int* __restrict__ list) {
    extern __shared__ int sh[];
    int* cnt = sh;
    int* base = sh + L;
    for (int q = threadIdx.x; q < L; q += blockDim.x) cnt[q] = 0;
    __syncthreads();
    for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += gridDim.x * blockDim.x) {  // uniform rounds
        const int i = i0 + threadIdx.x;
        int l = -1, pos = 0;
        if (i < n && cand[i].w > 1) {
            l = delta[i];
            pos = atomicAdd(&cnt[l], 1);
        }
        __syncthreads();
        for (int q = threadIdx.x; q < L; q += blockDim.x) {
            const int c = cnt[q];
            if (c) base[q] = atomicAdd(&cursor[q], c);
        }
        __syncthreads();
        if (l >= 0) list[base[l] + pos] = i;
        __syncthreads();
        for (int q = threadIdx.x; q < L; q += blockDim.x) cnt[q] = 0;
        __syncthreads();
    }
}

// Choice of a tied node i at level l: the candidate t with the smallest
// (key(t), t).  cand holds the first kMaxCand - 1 candidates and the count;
// with exactly kMaxCand candidates the last one is found by a scan from the
// third, with more every rank is scanned.
template <typename Key>
__device__ __forceinline__ int reg_pick(int n, int k, int l, int i, int4 c, const int* __restrict__ dist, Key key) {
    int pick = -1;
    long long pkey = 0;
    auto consider = [&](int t) {
        long long kk = ((long long)key(t) << 32) | t;
        if (pick < 0 || kk < pkey) {
            pick = t;
            pkey = kk;
        }
    };
    if (c.w <= kMaxCand) {
        consider(c.x);
        consider(c.y);
        if (c.w >= 3) consider(c.z);
        if (c.w == kMaxCand) {
            for (int t = c.z + 1; t < k; ++t)
                if (dist[(size_t)t * n + i] == l) {
                    consider(t);
                    break;
                }
        }
    } else {
        for (int t = 0; t < k; ++t)
            if (dist[(size_t)t * n + i] == l) consider(t);
    }
    return pick;
}

// Level-synchronous tie resolution in one workgroup (few tied nodes).
// cum[t] = region size from all levels below l; at level l the snapshot is
// cum[t] + U[t][l] (the single-candidate joins of level l); every tied node
// of level l takes the candidate with the smallest (snapshot, rank); then cum
// absorbs level l.  The result does not depend on the order of nodes inside
// a level.
__global__ __launch_bounds__(1024) void k_reg_resolve(int n, int k, int L, const int* __restrict__ dist,
                                                      const int* __restrict__ U,
                                                      const int* __restrict__ tstart,
                                                      const int* __restrict__ list,
                                                      const int4* __restrict__ cand,
                                                      int* __restrict__ region, int* cum, int* Tl) {
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        cum[t] = 0;
        Tl[t] = 0;
    }
    __syncthreads();
    for (int l = 0; l < L; ++l) {
        const int a = tstart[l], b = tstart[l + 1];
        for (int q = a + threadIdx.x; q < b; q += blockDim.x) {
            const int i = list[q];
            const int pick = reg_pick(n, k, l, i, cand[i], dist,
                                      [&](int t) { return cum[t] + U[(size_t)t * L + l]; });
            region[i] = pick;
            atomicAdd(&Tl[pick], 1);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < k; t += blockDim.x) {
            cum[t] += U[(size_t)t * L + l] + Tl[t];
            Tl[t] = 0;
        }
        __syncthreads();
    }
}

// Inclusive prefix of U over levels, in place: U[t][l] becomes the number of
// single-candidate nodes of region t at levels <= l.
__global__ void k_reg_ucum(int k, int L, int* __restrict__ U) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    int acc = 0;
    for (int l = 0; l < L; ++l) {
        acc += U[(size_t)t * L + l];
        U[(size_t)t * L + l] = acc;
    }
}

constexpr int kRegLdsMaxK = 8192;  // keys and counts of up to this many pivots in LDS

// One tied level l over many workgroups (the j-th level that has ties).
// With Ucum the inclusive level prefix of U, Tc_prev[t] the tied joins over
// the tied levels before the (j-1)-th and Tj[j-1][t] those of the (j-1)-th,
// the snapshot of level l is Ucum[t][l] + Tc_prev[t] + Tj[j-1][t]; workgroup
// 0 stores Tc_prev + Tj[j-1] into Tc_next for the next tied level (double
// buffer: launches on one stream run in order).  FULL scans every node for
// delta == l (coalesced distance reads when most nodes tie); otherwise the
// level's slice [a, b) of the tied-node list is processed.
template <bool FULL, bool LDS>
__global__ __launch_bounds__(256) void k_reg_level(int n, int k, int L, int l, int j, const int* __restrict__ dist,
                                                   const int* __restrict__ delta, const int4* __restrict__ cand,
                                                   const int* __restrict__ Ucum, const int* __restrict__ list, int a,
                                                   int b, const int* __restrict__ Tc_prev, int* __restrict__ Tc_next,
                                                   int* __restrict__ Tj, int* __restrict__ region) {
    extern __shared__ int sm[];  // LDS: key[k], cnt[k]
    int* key = sm;
    int* cnt = sm + k;
    const int* Tlast = j > 0 ? Tj + (size_t)(j - 1) * k : nullptr;
    int* Tcur = Tj + (size_t)j * k;
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        const int c = Tc_prev[t] + (Tlast ? Tlast[t] : 0);
        if (blockIdx.x == 0) Tc_next[t] = c;
        if (LDS) {
            key[t] = Ucum[(size_t)t * L + l] + c;
            cnt[t] = 0;
        }
    }
    __syncthreads();
    auto keyf = [&](int t) {
        if (LDS) return key[t];
        return Ucum[(size_t)t * L + l] + Tc_prev[t] + (Tlast ? Tlast[t] : 0);
    };
    auto one = [&](int i, int4 c) {
        const int pick = reg_pick(n, k, l, i, c, dist, keyf);
        region[i] = pick;
        if (LDS)
            atomicAdd(&cnt[pick], 1);
        else
            atomicAdd(&Tcur[pick], 1);
    };
    if (FULL) {
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            if (delta[i] != l) continue;
            const int4 c = cand[i];
            if (c.w > 1) one(i, c);
        }
    } else {
        for (int q = a + blockIdx.x * blockDim.x + threadIdx.x; q < b; q += gridDim.x * blockDim.x) {
            const int i = list[q];
            one(i, cand[i]);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int t = threadIdx.x; t < k; t += blockDim.x)
            if (cnt[t]) atomicAdd(&Tcur[t], cnt[t]);
    }
}

template <bool FULL>
static void launch_reg_level(int blocks, hipStream_t s, int n, int k, int L, int l, int j, const int* dist,
                             const int* delta, const int4* cand, const int* Ucum, const int* list, int a, int b,
                             const int* Tc_prev, int* Tc_next, int* Tj, int* region) {
    if (k <= kRegLdsMaxK)
        hipLaunchKernelGGL((k_reg_level<FULL, true>), dim3(blocks), dim3(256), sizeof(int) * 2 * (size_t)k, s, n, k,
                           L, l, j, dist, delta, cand, Ucum, list, a, b, Tc_prev, Tc_next, Tj, region);
    else
        hipLaunchKernelGGL((k_reg_level<FULL, false>), dim3(blocks), dim3(256), 0, s, n, k, L, l, j, dist, delta,
                           cand, Ucum, list, a, b, Tc_prev, Tc_next, Tj, region);
}

ssm_status regions(int32_t n, int32_t k, const int32_t* dist, int32_t* delta, int32_t* region,
                   hipStream_t s) {
    int4* cand = nullptr;
    int* aux = nullptr;
    ssm_status st = salloc((void**)&cand, sizeof(int4) * (size_t)n);
    if (st != SSM_OK) return st;
    st = salloc((void**)&aux, sizeof(int) * 2);
    if (st != SSM_OK) {
        sfree(cand);
        return st;
    }
    int grid = std::min(div_up(n, 256), 8192);
    int haux[2] = {0, 0};
    hipError_t e = hipMemsetAsync(aux, 0, sizeof(int) * 2, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_reg_scan, dim3(grid), dim3(256), 0, s, n, k, dist, delta, region, cand, aux);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(haux, aux, sizeof haux, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        sfree(cand);
        sfree(aux);
        return hip_fail(e, "region scan");
    }
    if (haux[1] > 0) {
        const int L = haux[0] + 1;
        // U[k][L], tcount[L], tstart[L+1], cursor[L], list[ntied], cum[k], Tl[k]
        size_t ints = (size_t)k * L + 3 * (size_t)L + 1 + (size_t)haux[1] + 2 * (size_t)k;
        int* ws = nullptr;
        st = salloc((void**)&ws, sizeof(int) * ints);
        if (st != SSM_OK) {
            sfree(cand);
            sfree(aux);
            return st;
        }
        int* U = ws;
        int* tcount = U + (size_t)k * L;
        int* tstart = tcount + L;
        int* cursor = tstart + L + 1;
        int* list = cursor + L;
        int* cum = list + haux[1];
        int* Tl = cum + k;
        // Few tied nodes: one workgroup walks the levels.  Many: one
        // multi-workgroup launch per level that has ties (tuning override
        // SSM_REGION_MODE: 1 one workgroup, 2 per level).
        const int mode = variant("region_mode");
        const bool per_level = mode == 2 || (mode != 1 && haux[1] > kRegOneWgMax);
        std::vector<int> hstart(L + 1);
        e = hipMemsetAsync(ws, 0, sizeof(int) * ((size_t)k * L + L), s);
        if (e == hipSuccess) {
            const long long hist_ints = (long long)(k + 1) * L;
            if (hist_ints <= kRegHistLds)
                hipLaunchKernelGGL(k_reg_hist<true>, dim3(std::min(grid, 4 * num_cus())), dim3(256),
                                   sizeof(int) * hist_ints, s, n, k, L, delta, cand, U, tcount);
            else
                hipLaunchKernelGGL(k_reg_hist<false>, dim3(grid), dim3(256), 0, s, n, k, L, delta, cand, U, tcount);
            hipLaunchKernelGGL(k_reg_prefix, dim3(1), dim3(64), 0, s, L, tcount, tstart, cursor);
            if (2LL * L <= kRegHistLds)
                hipLaunchKernelGGL(k_reg_scatter, dim3(std::min(grid, 4 * num_cus())), dim3(256),
                                   sizeof(int) * 2 * L, s, n, L, delta, cand, cursor, list);
            else
                hipLaunchKernelGGL(k_reg_scatter_global, dim3(grid), dim3(256), 0, s, n, delta, cand, cursor, list);
            if (!per_level)
                hipLaunchKernelGGL(k_reg_resolve, dim3(1), dim3(1024), 0, s, n, k, L, dist, U, tstart, list,
                                   cand, region, cum, Tl);
            e = hipGetLastError();
        }
        if (e == hipSuccess && per_level) {
            e = hipMemcpyAsync(hstart.data(), tstart, sizeof(int) * (L + 1), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            int nlev = 0;
            for (int l = 0; l < L; ++l) nlev += hstart[l + 1] > hstart[l];
            // Tc[2][k] double buffer, Tj[nlev][k]
            int* ws2 = nullptr;
            if (e == hipSuccess) {
                st = salloc((void**)&ws2, sizeof(int) * (size_t)k * (2 + nlev));
                if (st != SSM_OK) {  // the stream was synchronized above
                    sfree(ws);
                    sfree(cand);
                    sfree(aux);
                    return st;
                }
                e = hipMemsetAsync(ws2, 0, sizeof(int) * (size_t)k * (2 + nlev), s);
            }
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_reg_ucum, dim3(div_up(k, 256)), dim3(256), 0, s, k, L, U);
                int* Tc[2] = {ws2, ws2 + k};
                int* Tj = ws2 + 2 * (size_t)k;
                const int full_grid = std::min(div_up(n, 256), 4 * num_cus());
                int j = 0;
                for (int l = 0; l < L; ++l) {
                    const int a = hstart[l], b = hstart[l + 1];
                    if (b == a) continue;
                    const int* prev = Tc[j & 1];
                    int* next = Tc[(j + 1) & 1];
                    if ((long long)(b - a) * 16 >= n)
                        launch_reg_level<true>(full_grid, s, n, k, L, l, j, dist, delta, cand, U, list, a, b, prev,
                                               next, Tj, region);
                    else
                        launch_reg_level<false>(std::min(div_up(b - a, 256), 4 * num_cus()), s, n, k, L, l, j, dist,
                                                delta, cand, U, list, a, b, prev, next, Tj, region);
                    ++j;
                }
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (ws2) sfree(ws2);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipStreamSynchronize(s);  // idle before the scratch is reused (also after an error)
        sfree(ws);
    }
    (void)hipStreamSynchronize(s);
    sfree(cand);
    sfree(aux);
    if (e != hipSuccess) return hip_fail(e, "region assignment");
    return SSM_OK;
}

// ------------------------------------------------------------ layout pool

// Per graph (blockIdx.y): m = infinity, pivots = 0 (so that ranks a failed
// selection leaves unset still name a node), info = 0, and the padded
// adjacency of width kPoolEllW.
__global__ void k_pool_prep_init(const PoolGraph* __restrict__ gs) {
    const PoolGraph& g = gs[blockIdx.y];
    const int n = g.n;
    const long long ne = (long long)n * kPoolEllW;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < ne;
         q += (long long)gridDim.x * blockDim.x) {
        const int v = (int)(q / kPoolEllW), j = (int)(q % kPoolEllW);
        const int a = g.rp[v], d = g.rp[v + 1] - a;
        int val = -1;
        if (d > kPoolEllW && j == kPoolEllW - 1)
            val = kEllMore;
        else if (j < d)
            val = g.ci[a + j];
        g.ell[q] = val;
        if (j == 0) g.m[v] = kInf;
    }
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < max(g.kpad, 8); q += gridDim.x * blockDim.x) {
        if (q < g.kpad) g.pivots[q] = 0;
        if (q < 8) g.info[q] = 0;
    }
}

hipError_t pool_prep_init(const PoolGraph* gs, int count, int nmax, hipStream_t s) {
    const int bx = std::max(1, std::min(div_up((long long)nmax * kPoolEllW, 256), 256));
    hipLaunchKernelGGL(k_pool_prep_init, dim3(bx, count), dim3(256), 0, s, gs);
    return hipGetLastError();
}

// One max/min selection per graph, in one workgroup with LDS state bytes
// (LDS sized for the batch's largest graph; smaller pools let several
// selections share a CU).
constexpr int kPoolSelS = kLdsFixed + 22528, kPoolSelL = kLdsFixed + kPoolMaxN;
constexpr int kPoolSelBlock = 512;
constexpr int kPoolBfsBlock = 256;

template <int SPOOL>
__global__ __launch_bounds__(kPoolSelBlock) void k_pool_select(const PoolGraph* __restrict__ gs) {
    const PoolGraph& g = gs[blockIdx.x];
    select_ell_body<kPoolEllW, true, SPOOL>(g.n, g.rp, g.ci, g.ell, g.k, g.first, g.pivots, g.m, g.gq, g.info);
}

hipError_t pool_select(const PoolGraph* gs, int count, int nmax, hipStream_t s) {
    if (kLdsFixed + (((size_t)nmax + 15) & ~(size_t)15) <= (size_t)kPoolSelS)
        hipLaunchKernelGGL(k_pool_select<kPoolSelS>, dim3(count), dim3(kPoolSelBlock), 0, s, gs);
    else
        hipLaunchKernelGGL(k_pool_select<kPoolSelL>, dim3(count), dim3(kPoolSelBlock), 0, s, gs);
    return hipGetLastError();
}

// Items (graph, rank) over a persistent grid: the BFS from that graph's
// pivot of that rank into its distance row; info[1] = eccentricity maximum.
// Small workgroups: the pool's graphs have narrow frontiers, and several
// BFS then share a CU.
__global__ __launch_bounds__(kPoolBfsBlock) void k_pool_bfs(const PoolGraph* __restrict__ gs,
                                                            const int2* __restrict__ items, int nitems, int* gq,
                                                            long long gq_stride) {
    __shared__ int s_reached;
    int* myq = gq + (size_t)blockIdx.x * gq_stride;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 st = items[it];
        const PoolGraph& g = gs[st.x];
        __syncthreads();  // the previous item's last reads of LDS are done
        bfs_ell_body<kPoolEllW, kPoolS>(g.n, g.rp, g.ci, g.ell, g.pivots[st.y], g.dist + (size_t)st.y * g.n, myq,
                                         &s_reached, g.info + 1);
    }
}

int pool_bfs_blocks(int nitems) { return std::max(1, std::min(nitems, 5 * num_cus())); }

hipError_t pool_bfs(const PoolGraph* gs, const int2* items, int nitems, int* gq, long long gq_stride, int blocks,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_pool_bfs, dim3(blocks), dim3(kPoolBfsBlock), 0, s, gs, items, nitems, gq, gq_stride);
    return hipGetLastError();
}

}  // namespace ssm

extern "C" ssm_status ssm_validate_csr(const ssm_csr* g, hipStream_t stream) {
    using namespace ssm;
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    int* bad = nullptr;
    st = salloc((void**)&bad, sizeof(int));
    if (st != SSM_OK) return st;
    int hbad = 0;
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_validate_rows, dim3(std::min(div_up(g->n, 256), 8192)), dim3(256), 0, stream, g->n,
                           g->nnz, g->row_ptr, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess && hbad == 0 && g->nnz > 0) {  // the arcs' rows are in bounds only once the rows are valid
        hipLaunchKernelGGL(k_validate_arcs, dim3((int)std::min<long long>(div_up(g->nnz, 256), 16384)), dim3(256), 0,
                           stream, g->n, g->nnz, g->row_ptr, g->col_idx, bad);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    (void)hipStreamSynchronize(stream);
    sfree(bad);
    if (e != hipSuccess) return hip_fail(e, "CSR validation");
    if (hbad & 1) return fail(SSM_E_INVAL, "row_ptr is not monotone from 0 to nnz");
    if (hbad & 2) return fail(SSM_E_INVAL, "column index out of range or self-loop");
    if (hbad & 4) return fail(SSM_E_INVAL, "adjacency is not symmetric or has duplicate arcs");
    return SSM_OK;
}
