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
//
// Layout: the sums are feature-major, ST[j * k + t] = S_tj, so that the C
// sums one block needs for feature j are consecutive and wave-uniform: the
// contraction B = Y S^T (2 n k^2 flops per pass) runs as FP64 FMAs whose
// cluster operand comes from scalar loads, one node per lane, C clusters
// per block.  Every product and partial sum is an integer below 2^53, so the
// FMAs are exact in any order.
#include <stdlib.h>

#include <climits>
#include <vector>

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

constexpr int kKmBlock = 256;
constexpr int kKmChunk = 32;   // clusters per block of the nearest-node kernel
constexpr int kKmPad = 64;     // zero doubles after the sums: the widest chunk may read that far past row k-1
constexpr int kKmMaxK = 4096;  // the sums' partial tables are (k + 1) k words per node range
constexpr int kKmMinBlocks = 2048;
constexpr int kKmReduceSlice = 8;  // partial tables summed per thread before one atomic add

// ST (k k doubles, then kKmPad zero doubles so that a block's last chunk
// may read past row k-1), N, and assign = -1 (no cluster yet).
__global__ void k_km_init(int n, int k, const int* __restrict__ dist, const int* __restrict__ pivots,
                          double* __restrict__ ST, double* __restrict__ N, int* __restrict__ assign) {
    const long long kk = (long long)k * k, total = kk + kKmPad + n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        if (q < kk) {
            const int j = (int)(q / k), t = (int)(q % k);
            ST[q] = (double)dist[(size_t)j * n + pivots[t]];
            if (j == 0) N[t] = 1.0;
        } else if (q < kk + kKmPad) {
            ST[q] = 0.0;
        } else {
            assign[q - kk - kKmPad] = -1;
        }
    }
}

// ||y_i||^2 as a 64-bit integer.
__global__ void k_km_norm(int n, int k, const int* __restrict__ dist, long long* __restrict__ q) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long long s = 0;
    for (int j = 0; j < k; ++j) {
        const long long y = dist[(size_t)j * n + i];
        s += y * y;
    }
    q[i] = s;
}

// a_t = sum_j (S_tj / N_t)^2, ascending j, each quotient, square and sum
// rounded: one block per t squares 256 features at a time in parallel, one
// lane adds them in order.
__global__ __launch_bounds__(256) void k_km_a(int k, const double* __restrict__ ST, const double* __restrict__ N,
                                              double* __restrict__ a) {
#pragma clang fp contract(off)
    __shared__ double sq[256];
    const int t = blockIdx.x;
    const double nt = N[t];
    double s = 0.0;
    for (int j0 = 0; j0 < k; j0 += 256) {
        const int j = j0 + threadIdx.x;
        if (j < k) {
            const double c = ST[(size_t)j * k + t] / nt;
            sq[threadIdx.x] = c * c;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int u = 0; u < min(256, k - j0); ++u) s += sq[u];
        __syncthreads();
    }
    if (threadIdx.x == 0) a[t] = s;
}

// b[c] = B_{t0+c, i} = sum_j y_ij S_{t0+c, j} for c < C (columns at or past
// k read the zero padding or the next row: finite, never used).  One
// feature's C sums are wave-uniform loads.
template <int C>
__device__ __forceinline__ void km_contract(int n, int k, int i, int t0, const int* __restrict__ dist,
                                            const double* __restrict__ ST, double (&b)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) b[c] = 0.0;
    const int* yp = dist + i;
    const double* sp = ST + t0;
    int j = 0;
    int yn[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) yn[u] = yp[(size_t)min(u, k - 1) * n];
    for (; j + 4 <= k; j += 4) {
        double y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = (double)yn[u];
#pragma unroll
        for (int u = 0; u < 4; ++u) yn[u] = yp[(size_t)min(j + 4 + u, k - 1) * n];  // next group, clamped in range
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double* row = sp + (size_t)(j + u) * k;
#pragma unroll
            for (int c = 0; c < C; ++c) b[c] = __builtin_fma(y[u], row[c], b[c]);
        }
    }
    for (int u = 0; j < k; ++j, ++u) {
        const double y = (double)yn[u];
        const double* row = sp + (size_t)j * k;
#pragma unroll
        for (int c = 0; c < C; ++c) b[c] = __builtin_fma(y, row[c], b[c]);
    }
}

// Assignment, one chunk of C clusters per blockIdx.y: the first t of the
// chunk with the smallest f_t(i) goes to fb/tb[chunk][i].
template <int C>
__global__ __launch_bounds__(kKmBlock) void k_km_assign(int n, int k, const int* __restrict__ dist,
                                                        const double* __restrict__ ST, const double* __restrict__ N,
                                                        const double* __restrict__ a, double* __restrict__ fb,
                                                        int* __restrict__ tb) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t0 = blockIdx.y * C;
    const int ct = min(C, k - t0);
    double b[C];
    km_contract<C>(n, k, i, t0, dist, ST, b);
    int best = t0;
    double fbest = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (c < ct) {
            const int t = t0 + c;
            const double f = a[t] - (2.0 * b[c]) / N[t];
            if (c == 0 || f < fbest) {
                best = t;
                fbest = f;
            }
        }
    }
    fb[(size_t)blockIdx.y * n + i] = fbest;
    tb[(size_t)blockIdx.y * n + i] = best;
}

// Chunks in ascending order, strict improvement only: the lowest t with the
// smallest f.  changed[0] counts moved nodes.
__global__ __launch_bounds__(kKmBlock) void k_km_pick(int n, int nchunks, const double* __restrict__ fb,
                                                      const int* __restrict__ tb, int* __restrict__ assign,
                                                      int* changed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool moved = false;
    if (i < n) {
        double fbest = fb[i];
        int best = tb[i];
        for (int c = 1; c < nchunks; ++c) {
            const double f = fb[(size_t)c * n + i];
            if (f < fbest) {
                fbest = f;
                best = tb[(size_t)c * n + i];
            }
        }
        moved = assign[i] != best;
        assign[i] = best;
    }
    const unsigned long long m = __ballot(moved);
    if (lane_id() == 0 && m) atomicAdd(changed, (int)__popcll(m));
}

// Member sums of `rows` feature rows (row k = member counts) over nodes
// [bx span, (bx+1) span): LDS 64-bit counters, one add per wave when the
// whole wave shares a cluster, else one per node.  Each block writes its
// partial table part[bx][j0 .. j0+rows)[k].
__global__ __launch_bounds__(kKmBlock) void k_km_sums(int n, int k, int rows_per_block, int span,
                                                      const int* __restrict__ dist, const int* __restrict__ assign,
                                                      unsigned long long* __restrict__ part) {
    extern __shared__ unsigned long long acc[];  // [rows_per_block][k]
    const int j0 = blockIdx.y * rows_per_block;
    const int rows = min(rows_per_block, k + 1 - j0);
    for (int q = threadIdx.x; q < rows * k; q += blockDim.x) acc[q] = 0;
    __syncthreads();
    const int i0 = blockIdx.x * span, i1 = min(n, i0 + span);
    for (int base = i0; base < i1; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const bool ok = i < i1;
        const int t = ok ? assign[i] : 0;
        const int tf = __builtin_amdgcn_readfirstlane(t);
        const bool uniform = __ballot(!ok || t != tf) == 0;
        for (int r = 0; r < rows; ++r) {
            const int j = j0 + r;
            long long v = 0;
            if (ok) v = j < k ? (long long)dist[(size_t)j * n + i] : 1;
            if (uniform) {
                v = wave_sum(v);
                if (lane_id() == 0) atomicAdd(&acc[r * k + tf], (unsigned long long)v);
            } else if (ok) {
                atomicAdd(&acc[r * k + t], (unsigned long long)v);
            }
        }
    }
    __syncthreads();
    unsigned long long* out = part + (size_t)blockIdx.x * (k + 1) * k + (size_t)j0 * k;
    for (int q = threadIdx.x; q < rows * k; q += blockDim.x) out[q] = acc[q];
}

// S2 (zeroed) += the partial tables of blocks [y slice, (y+1) slice).
__global__ void k_km_reduce(int nbx, int slice, int k, const unsigned long long* __restrict__ part,
                            unsigned long long* __restrict__ S2) {
    const long long w = (long long)(k + 1) * k;
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= w) return;
    const int b0 = blockIdx.y * slice, b1 = min(nbx, b0 + slice);
    unsigned long long s = 0;
    for (int bx = b0; bx < b1; ++bx) s += part[(size_t)bx * w + q];
    if (s) atomicAdd(&S2[q], s);
}

// Non-empty clusters take their new sums; an empty one keeps its centroid.
__global__ void k_km_commit(int k, const unsigned long long* __restrict__ S2, double* __restrict__ ST,
                            double* __restrict__ N) {
    const long long kk = (long long)k * k;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < kk;
         q += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(q / k), t = (int)(q % k);
        const unsigned long long cnt = S2[kk + t];
        if (cnt > 0) {
            ST[q] = (double)S2[q];
            if (j == 0) N[t] = (double)cnt;
        }
    }
}

__device__ __forceinline__ void km_argmin_pair(long long& s, int& id, long long s2, int id2) {
    if (s2 < s || (s2 == s && id2 < id)) {
        s = s2;
        id = id2;
    }
}

// Nearest free node to each of C centroids t_base + blockIdx.y C + c over
// this block's nodes: smallest N_t q_i - 2 B_ti, then lowest id; one
// (score, node) pair per (block, t) into ps/pn[bx][t].
template <int C>
__global__ __launch_bounds__(kKmBlock) void k_km_near(int n, int k, int t_base, const int* __restrict__ dist,
                                                      const double* __restrict__ ST, const double* __restrict__ N,
                                                      const long long* __restrict__ q,
                                                      const unsigned char* __restrict__ taken,
                                                      long long* __restrict__ ps, int* __restrict__ pn) {
    __shared__ long long ws[kKmBlock / kWave][C];
    __shared__ int wn[kKmBlock / kWave][C];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int t0 = t_base + blockIdx.y * C;
    const int ct = min(C, k - t0);
    double b[C];
    const bool live = i < n && !taken[i];
    if (i < n) km_contract<C>(n, k, i, t0, dist, ST, b);
    const long long qi = live ? q[i] : 0;
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (c < ct) {
            long long s = LLONG_MAX;
            int id = INT_MAX;
            if (live) {
                s = (long long)N[t0 + c] * qi - 2 * (long long)b[c];
                id = i;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) km_argmin_pair(s, id, __shfl_xor(s, off), __shfl_xor(id, off));
            if (lane_id() == 0) {
                ws[w][c] = s;
                wn[w][c] = id;
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < ct) {
        const int c = threadIdx.x;
        long long s = ws[0][c];
        int id = wn[0][c];
        for (int u = 1; u < kKmBlock / kWave; ++u) km_argmin_pair(s, id, ws[u][c], wn[u][c]);
        ps[(size_t)blockIdx.x * k + t0 + c] = s;
        pn[(size_t)blockIdx.x * k + t0 + c] = id;
    }
}

// One block per t: the (score, node) minimum over the nbx block results.
__global__ __launch_bounds__(256) void k_km_near_reduce(int nbx, int k, int t_base, const long long* __restrict__ ps,
                                                        const int* __restrict__ pn, int* __restrict__ node) {
    __shared__ long long ws[256 / kWave];
    __shared__ int wn[256 / kWave];
    const int t = t_base + blockIdx.x;
    long long s = LLONG_MAX;
    int id = INT_MAX;
    for (int bx = threadIdx.x; bx < nbx; bx += blockDim.x)
        km_argmin_pair(s, id, ps[(size_t)bx * k + t], pn[(size_t)bx * k + t]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) km_argmin_pair(s, id, __shfl_xor(s, off), __shfl_xor(id, off));
    if (lane_id() == 0) {
        ws[threadIdx.x / kWave] = s;
        wn[threadIdx.x / kWave] = id;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int u = 1; u < 256 / kWave; ++u) km_argmin_pair(s, id, ws[u], wn[u]);
        node[t] = id == INT_MAX ? -1 : id;
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

namespace {

hipError_t km_nearest(int n, int k, int t_base, int t_count, const int* dist, const double* ST, const double* N,
                      const long long* q, const unsigned char* taken, long long* ps, int* pn, int* node,
                      hipStream_t s) {
    const int nb = div_up(n, kKmBlock);
    if (t_count == 1) {
        hipLaunchKernelGGL(k_km_near<1>, dim3(nb, 1), dim3(kKmBlock), 0, s, n, k, t_base, dist, ST, N, q, taken, ps,
                           pn);
    } else {
        hipLaunchKernelGGL(k_km_near<kKmChunk>, dim3(nb, div_up(t_count, kKmChunk)), dim3(kKmBlock), 0, s, n, k,
                           t_base, dist, ST, N, q, taken, ps, pn);
    }
    hipLaunchKernelGGL(k_km_near_reduce, dim3(t_count), dim3(256), 0, s, nb, k, t_base, ps, pn, node);
    return hipGetLastError();
}

}  // namespace

ssm_status kmeans_pivots(int32_t n, int32_t k, const int32_t* pivots, const int32_t* dist, int32_t max_iters,
                         int32_t* new_pivots, int32_t* assign_out, int32_t* iters_host, hipStream_t s) {
    if (k > kKmMaxK) return fail(SSM_E_RANGE, "k-means sp: k above 4096");
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
    // launch shapes
    const int nb = div_up(n, kKmBlock);
    // assignment chunk: fewest padded clusters, each chunk costing about 8
    // more for its re-read of the distance table
    int C = 0, cost = INT_MAX;
    for (int c : {32, 40, 48, 56, 64}) {
        const int cc = div_up(k, c) * (c + 8);
        if (cc < cost) {
            cost = cc;
            C = c;
        }
    }
    if (const int c = variant("km_chunk")) {
        if (c == 32 || c == 40 || c == 48 || c == 56 || c == 64) C = c;
    }
    const int nchunks = div_up(k, C);
    auto assign_kernel = C == 32 ? k_km_assign<32> : C == 40 ? k_km_assign<40> : C == 48 ? k_km_assign<48>
                       : C == 56 ? k_km_assign<56> : k_km_assign<64>;
    const int rows_per_block = std::max(1, std::min(8, 4096 / k));  // LDS: rows k 8 bytes <= 32 KB
    const int ny = div_up(k + 1, rows_per_block);
    int nbx = std::max(1, std::min(nb, div_up(kKmMinBlocks, ny)));
    const int span = div_up(div_up(n, nbx), kKmBlock) * kKmBlock;
    nbx = div_up(n, span);
    // workspace
    const size_t kk = (size_t)k * k, w = (size_t)(k + 1) * k;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_st = take(sizeof(double) * (kk + kKmPad)), o_n = take(sizeof(double) * k),
                 o_a = take(sizeof(double) * k), o_q = take(sizeof(long long) * n),
                 o_fb = take(sizeof(double) * (size_t)nchunks * n), o_tb = take(sizeof(int) * (size_t)nchunks * n),
                 o_as = take(sizeof(int) * (size_t)n), o_ch = take(sizeof(int)),
                 o_part = take(sizeof(unsigned long long) * (size_t)nbx * w), o_s2 = take(sizeof(unsigned long long) * w),
                 o_ps = take(sizeof(long long) * (size_t)nb * k), o_pn = take(sizeof(int) * (size_t)nb * k),
                 o_tk = take((size_t)n), o_nd = take(sizeof(int) * k);
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, off);
    if (st != SSM_OK) return st;
    double* ST = (double*)(ws + o_st);
    double* N = (double*)(ws + o_n);
    double* a = (double*)(ws + o_a);
    long long* q = (long long*)(ws + o_q);
    double* fb = (double*)(ws + o_fb);
    int* tb = (int*)(ws + o_tb);
    int* assign = assign_out ? assign_out : (int*)(ws + o_as);
    int* changed = (int*)(ws + o_ch);
    unsigned long long* part = (unsigned long long*)(ws + o_part);
    unsigned long long* S2 = (unsigned long long*)(ws + o_s2);
    long long* ps = (long long*)(ws + o_ps);
    int* pn = (int*)(ws + o_pn);
    unsigned char* taken = (unsigned char*)(ws + o_tk);
    int* nodes = (int*)(ws + o_nd);

    const int grid_init = std::max(1, std::min(div_up((long long)kk + kKmPad + n, 256), 8192));
    hipLaunchKernelGGL(k_km_init, dim3(grid_init), dim3(256), 0, s, n, k, dist, pivots, ST, N, assign);
    hipLaunchKernelGGL(k_km_norm, dim3(nb), dim3(kKmBlock), 0, s, n, k, dist, q);
    hipError_t e = hipGetLastError();
    int it = 0;
    while (e == hipSuccess && it < max_iters) {
        ++it;
        hipLaunchKernelGGL(k_km_a, dim3(k), dim3(256), 0, s, k, ST, N, a);
        e = hipMemsetAsync(changed, 0, sizeof(int), s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(assign_kernel, dim3(nb, nchunks), dim3(kKmBlock), 0, s, n, k, dist, ST, N, a, fb, tb);
        hipLaunchKernelGGL(k_km_pick, dim3(nb), dim3(kKmBlock), 0, s, n, nchunks, fb, tb, assign, changed);
        hipLaunchKernelGGL(k_km_sums, dim3(nbx, ny), dim3(kKmBlock),
                           sizeof(unsigned long long) * (size_t)rows_per_block * k, s, n, k, rows_per_block, span,
                           dist, assign, part);
        e = hipMemsetAsync(S2, 0, sizeof(unsigned long long) * w, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_km_reduce, dim3(div_up((long long)w, 256), div_up(nbx, kKmReduceSlice)), dim3(256), 0, s,
                           nbx, kKmReduceSlice, k, part, S2);
        hipLaunchKernelGGL(k_km_commit, dim3(std::max(1, std::min(div_up((long long)kk, 256), 4096))), dim3(256), 0, s,
                           k, S2, ST, N);
        e = hipGetLastError();
        int hchanged = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&hchanged, changed, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess || hchanged == 0) break;
    }
    // nearest free node per cluster: all clusters at once, then each one
    // whose choice a lower rank already took again, without the taken nodes
    std::vector<int> hnodes(k);
    if (e == hipSuccess) e = hipMemsetAsync(taken, 0, (size_t)n, s);
    if (e == hipSuccess) e = km_nearest(n, k, 0, k, dist, ST, N, q, taken, ps, pn, nodes, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hnodes.data(), nodes, sizeof(int) * k, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    std::vector<int> result(k, -1);
    std::vector<unsigned char> used;
    if (e == hipSuccess) used.assign((size_t)n, 0);
    for (int t = 0; t < k && e == hipSuccess; ++t) {
        int v = hnodes[t];
        if (v < 0 || used[v]) {
            e = hipMemcpyAsync(taken, used.data(), (size_t)n, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = km_nearest(n, k, t, 1, dist, ST, N, q, taken, ps, pn, nodes, s);
            if (e == hipSuccess) e = hipMemcpyAsync(&v, nodes + t, sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) break;
            if (v < 0) {  // cannot happen: fewer than k nodes are taken
                e = hipErrorUnknown;
                break;
            }
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
