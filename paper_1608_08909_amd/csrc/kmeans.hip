// k-means sp pivot refinement (paper Section 4.1, "k-means sp"): Lloyd
// iterations over the nodes' hop-distance vectors to the max/min pivots.
//
// Node i's feature vector is y_i = (dist[0][i], ..., dist[k-1][i]).  Cluster
// t is held as the exact integer sum S_t of its members' vectors (in double:
// every sum stays below 2^53) and its size N_t; it starts as y_{p_t}.  One
// pass: every node joins the cluster with the smallest
//     f_t(i) = a_t - (2 B_ti) / N_t,   B_ti = y_i . S_t (an exact integer),
//     a_t = sum_j (S_tj / N_t)^2 in ascending j, no fused multiply-add,
// lowest t on ties; every non-empty cluster's sums are then recomputed (an
// empty one keeps its centroid).  Passes stop when no node moves or after
// max_iters.  New pivot t is the free node with the smallest
// N_t ||y_i||^2 - 2 B_ti (exact 64-bit integers), lowest id on ties, ranks in
// ascending order.
#include <stdlib.h>

#include <vector>

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

constexpr int kKmBlock = 256;
constexpr int kKmChunk = 32;  // most clusters per pass of the assignment kernel
constexpr int kKmMaxK = 16384;  // one cluster's sums (8 k bytes) fit in LDS

__global__ void k_km_init(int n, int k, const int* __restrict__ dist, const int* __restrict__ pivots,
                          double* __restrict__ S, double* __restrict__ N, int* __restrict__ assign) {
    const long long kk = (long long)k * k;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < kk + n;
         q += (long long)gridDim.x * blockDim.x) {
        if (q < kk) {
            const int t = (int)(q / k), j = (int)(q % k);
            S[q] = (double)dist[(size_t)j * n + pivots[t]];
            if (j == 0) N[t] = 1.0;
        } else {
            assign[q - kk] = -1;
        }
    }
}

// a_t = sum_j (S_tj / N_t)^2, ascending j, each product and sum rounded.
__global__ void k_km_a(int k, const double* __restrict__ S, const double* __restrict__ N, double* __restrict__ a) {
#pragma clang fp contract(off)
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k; t += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) {
            const double c = S[(size_t)t * k + j] / N[t];
            s += c * c;
        }
        a[t] = s;
    }
}

// One thread per node: B_ti for kKmChunk clusters at a time (their sums in
// LDS), then f_t(i); argmin over all t.  changed[0] counts moved nodes.
__global__ __launch_bounds__(kKmBlock) void k_km_assign(int n, int k, const int* __restrict__ dist,
                                                        const double* __restrict__ S, const double* __restrict__ N,
                                                        const double* __restrict__ a, int cmax,
                                                        int* __restrict__ assign, int* changed) {
#pragma clang fp contract(off)
    extern __shared__ double sS[];  // [cmax][k], cmax <= kKmChunk
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int best = 0;
    double fbest = 0.0;
    for (int t0 = 0; t0 < k; t0 += cmax) {
        const int ct = min(cmax, k - t0);
        __syncthreads();
        for (int q = threadIdx.x; q < ct * k; q += blockDim.x) sS[q] = S[(size_t)t0 * k + q];
        __syncthreads();
        if (i < n) {
            double b[kKmChunk];
#pragma unroll
            for (int c = 0; c < kKmChunk; ++c) b[c] = 0.0;
            for (int j = 0; j < k; ++j) {
                const double y = (double)dist[(size_t)j * n + i];
#pragma unroll
                for (int c = 0; c < kKmChunk; ++c)
                    if (c < ct) b[c] = __builtin_fma(y, sS[c * k + j], b[c]);  // exact: integers below 2^53
            }
            for (int c = 0; c < ct; ++c) {
                const int t = t0 + c;
                const double f = a[t] - (2.0 * b[c]) / N[t];
                if (t == 0 || f < fbest) {
                    best = t;
                    fbest = f;
                }
            }
        }
    }
    if (i < n) {
        if (assign[i] != best) atomicAdd(changed, 1);
        assign[i] = best;
    }
}

// New member sums: thread per (feature j, node i), j-major (coalesced
// reads of dist rows); double atomics on integers are exact in any order.
__global__ void k_km_sums(int n, int k, const int* __restrict__ dist, const int* __restrict__ assign,
                          double* __restrict__ S2, double* __restrict__ N2) {
    const long long total = (long long)k * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(q / n), i = (int)(q % n);
        const int t = assign[i];
        atomicAdd(&S2[(size_t)t * k + j], (double)dist[q]);
        if (j == 0) atomicAdd(&N2[t], 1.0);
    }
}

// Non-empty clusters take their new sums; an empty one keeps its centroid.
__global__ void k_km_commit(int k, const double* __restrict__ S2, const double* __restrict__ N2,
                            double* __restrict__ S, double* __restrict__ N) {
    const long long kk = (long long)k * k;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < kk;
         q += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(q / k);
        if (N2[t] > 0.0) {
            S[q] = S2[q];
            if (q % k == 0) N[t] = N2[t];
        }
    }
}

// Block b handles cluster t = tlist[b]: argmin over free nodes of
// N_t ||y_i||^2 - 2 B_ti (64-bit integers), lowest id on ties.
__global__ __launch_bounds__(kKmBlock) void k_km_nearest(int n, int k, const int* __restrict__ dist,
                                                         const double* __restrict__ S, const double* __restrict__ N,
                                                         const int* __restrict__ tlist,
                                                         const unsigned char* __restrict__ taken,
                                                         long long* __restrict__ out_score, int* __restrict__ out_node) {
    extern __shared__ double sc[];  // centroid sums of this cluster [k]
    const int t = tlist[blockIdx.x];
    for (int j = threadIdx.x; j < k; j += blockDim.x) sc[j] = S[(size_t)t * k + j];
    __syncthreads();
    const long long nt = (long long)N[t];
    long long bs = 0;
    int bi = -1;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {  // ascending per thread
        if (taken[i]) continue;
        long long q = 0, b = 0;
        for (int j = 0; j < k; ++j) {
            const long long y = dist[(size_t)j * n + i];
            q += y * y;
            b += y * (long long)sc[j];
        }
        const long long s = nt * q - 2 * b;
        if (bi < 0 || s < bs) {
            bs = s;
            bi = i;
        }
    }
    __shared__ long long rs[kKmBlock];
    __shared__ int ri[kKmBlock];
    rs[threadIdx.x] = bs;
    ri[threadIdx.x] = bi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const long long s2 = rs[threadIdx.x + w];
            const int i2 = ri[threadIdx.x + w];
            const bool better = i2 >= 0 && (ri[threadIdx.x] < 0 || s2 < rs[threadIdx.x] ||
                                            (s2 == rs[threadIdx.x] && i2 < ri[threadIdx.x]));
            if (better) {
                rs[threadIdx.x] = s2;
                ri[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_score[blockIdx.x] = rs[0];
        out_node[blockIdx.x] = ri[0];
    }
}

// Largest entry of dist (block maxima, one atomic per block).
__global__ __launch_bounds__(256) void k_km_dmax(long long total, const int* __restrict__ dist, int* out) {
    int m = 0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x)
        m = max(m, dist[q]);
    __shared__ int red[256 / kWave];
    m = block_max(m, red);
    if (threadIdx.x == 0) atomicMax(out, m);
}

ssm_status kmeans_pivots(int32_t n, int32_t k, const int32_t* pivots, const int32_t* dist, int32_t max_iters,
                         int32_t* new_pivots, int32_t* assign_out, int32_t* iters_host, hipStream_t s) {
    if (k > kKmMaxK) return fail(SSM_E_RANGE, "k-means sp: k above 16384");
    {  // the pivots index the distance rows' columns
        std::vector<int> hp(k);
        hipError_t e0 = hipMemcpyAsync(hp.data(), pivots, sizeof(int) * k, hipMemcpyDeviceToHost, s);
        if (e0 == hipSuccess) e0 = hipStreamSynchronize(s);
        if (e0 != hipSuccess) return hip_fail(e0, "k-means sp: pivots");
        for (int t = 0; t < k; ++t)
            if (hp[t] < 0 || hp[t] >= n) return fail(SSM_E_INVAL, "k-means sp: pivot out of range");
    }
    {  // every product and sum of the exact integer arithmetic stays below 2^53
        int* dm = nullptr;
        ssm_status st0 = salloc((void**)&dm, sizeof(int));
        if (st0 != SSM_OK) return st0;
        int hdm = 0;
        hipError_t e0 = hipMemsetAsync(dm, 0, sizeof(int), s);
        if (e0 == hipSuccess) {
            hipLaunchKernelGGL(k_km_dmax, dim3(std::max(1, std::min(div_up((long long)k * n, 256), 4096))), dim3(256),
                               0, s, (long long)k * n, dist, dm);
            e0 = hipGetLastError();
        }
        if (e0 == hipSuccess) e0 = hipMemcpyAsync(&hdm, dm, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e0 == hipSuccess) e0 = hipStreamSynchronize(s);
        (void)hipStreamSynchronize(s);
        sfree(dm);
        if (e0 != hipSuccess) return hip_fail(e0, "k-means sp: distance range");
        if ((double)k * (double)n * (double)hdm * (double)hdm >= 9007199254740992.0)
            return fail(SSM_E_RANGE, "k-means sp: k * n * dmax^2 reaches 2^53 (exact integer sums not guaranteed)");
    }
    // doubles: S, S2 [k][k]; N, N2, a [k]; ints: assign [n], changed, tlist [k],
    // nodes [k]; long longs: scores [k]; bytes: taken [n]
    const size_t kk = (size_t)k * k;
    const size_t bytes = sizeof(double) * (2 * kk + 3 * (size_t)k) + sizeof(int) * ((size_t)n + 1 + 2 * (size_t)k) +
                         sizeof(long long) * (size_t)k + (size_t)n + 64;
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, bytes);
    if (st != SSM_OK) return st;
    double* S = (double*)ws;
    double* S2 = S + kk;
    double* N2 = S2 + kk;  // right after S2: one clear covers both
    double* N = N2 + k;
    double* a = N + k;
    long long* scores = (long long*)(a + k);
    int* assign = assign_out ? assign_out : (int*)(scores + k);
    int* changed = (int*)(scores + k) + n;
    int* tlist = changed + 1;
    int* nodes = tlist + k;
    unsigned char* taken = (unsigned char*)(nodes + k);
    const int grid_kk = std::max(1, std::min(div_up((long long)kk + n, 256), 8192));
    hipLaunchKernelGGL(k_km_init, dim3(grid_kk), dim3(256), 0, s, n, k, dist, pivots, S, N, assign);
    hipError_t e = hipGetLastError();
    const int nb = div_up(n, kKmBlock);
    const int cmax = std::max(1, std::min(kKmChunk, (int)(64 * 1024 / (sizeof(double) * (size_t)k))));
    const size_t lds = sizeof(double) * cmax * (size_t)k;  // at most 128 KB
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void*)k_km_assign, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void*)k_km_nearest, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    int it = 0;
    while (e == hipSuccess && it < max_iters) {
        ++it;
        hipLaunchKernelGGL(k_km_a, dim3(div_up(k, 64)), dim3(64), 0, s, k, S, N, a);
        e = hipMemsetAsync(changed, 0, sizeof(int), s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_km_assign, dim3(nb), dim3(kKmBlock), lds, s, n, k, dist, S, N, a, cmax, assign,
                           changed);
        e = hipMemsetAsync(S2, 0, sizeof(double) * (kk + k), s);  // S2 and N2 are adjacent
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_km_sums, dim3(std::min(div_up((long long)k * n, 256), 16384)), dim3(256), 0, s, n, k, dist,
                           assign, S2, N2);
        hipLaunchKernelGGL(k_km_commit, dim3(std::max(1, std::min(div_up((long long)kk, 256), 4096))), dim3(256), 0, s,
                           k, S2, N2, S, N);
        e = hipGetLastError();
        int hchanged = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&hchanged, changed, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess || hchanged == 0) break;
    }
    // nearest free node per cluster: all clusters at once, then the ones
    // whose choice collides with a lower rank again, one by one
    std::vector<int> hnodes(k), order(k);
    if (e == hipSuccess) e = hipMemsetAsync(taken, 0, (size_t)n, s);
    for (int t = 0; t < k; ++t) order[t] = t;
    if (e == hipSuccess) e = hipMemcpyAsync(tlist, order.data(), sizeof(int) * k, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_km_nearest, dim3(k), dim3(kKmBlock), sizeof(double) * (size_t)k, s, n, k, dist, S, N,
                           tlist, taken, scores, nodes);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hnodes.data(), nodes, sizeof(int) * k, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    std::vector<int> result(k, -1);
    std::vector<unsigned char> used;
    if (e == hipSuccess) used.assign((size_t)n, 0);
    for (int t = 0; t < k && e == hipSuccess; ++t) {
        int v = hnodes[t];
        if (v < 0 || used[v]) {  // taken by a lower rank: search again without the taken nodes
            e = hipMemcpyAsync(taken, used.data(), (size_t)n, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(tlist, &t, sizeof(int), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_km_nearest, dim3(1), dim3(kKmBlock), sizeof(double) * (size_t)k, s, n, k, dist,
                                   S, N, tlist, taken, scores, nodes);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipMemcpyAsync(&v, nodes, sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) break;
        }
        result[t] = v;
        used[v] = 1;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(new_pivots, result.data(), sizeof(int) * k, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "k-means sp");
    if (iters_host) *iters_host = it;
    return SSM_OK;
}

}  // namespace ssm
