// Term set of the sparse stress model: region histograms, adapted weights
// w'_ip = s / d_ip^2 and the denominators of Eq. 5 (paper Section 3).
#include <limits.h>

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

// Whether the FP32 sweep's node order can pay: aux[2] = largest degree;
// over the first kLocalSample arcs of every row, aux[3] = those whose ends
// lie at most kLocalSpan ids apart (64 KB of FP32 coordinates) and aux[4]
// = all of them.
constexpr int kLocalSpan = 8192;
constexpr int kLocalSample = 32;
__global__ __launch_bounds__(256) void k_order_stats(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     int* aux) {
    int dmax = 0, local = 0, seen = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int a = rp[i], b = rp[i + 1];
        dmax = max(dmax, b - a);
        const int c = min(b, a + kLocalSample);
        for (int e = a; e < c; ++e) local += abs(ci[e] - i) <= kLocalSpan;
        seen += c - a;
    }
    __shared__ int red[256 / kWave];
    dmax = block_max(dmax, red);
    local = block_sum(local, red);
    seen = block_sum(seen, red);
    if (threadIdx.x == 0) {  // one atomic per word and block
        atomicMax(&aux[2], dmax);
        atomicAdd(&aux[3], local);
        atomicAdd(&aux[4], seen);
    }
}

// aux[0] = max delta, aux[1] = max dist.
__global__ __launch_bounds__(256) void k_terms_max(int n, int k, const int* __restrict__ dist, const int* __restrict__ delta,
                            int* aux) {
    int dm = 0, mx = 0;
    long long total = (long long)k * n;
    const long long stride = (long long)gridDim.x * blockDim.x;
    // 16-byte loads, four in flight, when the caller's table is 16-byte
    // aligned; the rest (or all of it) one int at a time
    const long long n4 = ((uintptr_t)dist & 15) == 0 ? total / 4 : 0;
    const int4* d4 = (const int4*)dist;
    for (long long q0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; q0 < n4; q0 += 4 * stride) {
        int4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = q0 + j * stride < n4 ? d4[q0 + j * stride] : make_int4(0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) mx = max(mx, max(max(v[j].x, v[j].y), max(v[j].z, v[j].w)));
    }
    for (long long q = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total; q += stride)
        mx = max(mx, dist[q]);
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += stride) {
        const int a = delta[q];
        dm = a > dm ? a : dm;
    }
    __shared__ int red[256 / kWave];
    dm = block_max(dm, red);
    mx = block_max(mx, red);
    if (threadIdx.x == 0) {  // one atomic per block
        atomicMax(&aux[0], dm);
        atomicMax(&aux[1], mx);
    }
}

// Raw histogram of (region, delta), then a per-pivot running sum over the
// level: H[t][l] = |{ j : region_j = t, delta_j <= l }|.
// With LDS the block counts into LDS (k L counters) and adds its nonzero
// counts to H at the end.
template <bool LDS>
__global__ __launch_bounds__(256) void k_terms_hist(int n, int k, int L, const int* __restrict__ delta,
                                                    const int* __restrict__ region, int* __restrict__ H) {
    extern __shared__ int sh[];
    if (LDS) {
        for (int q = threadIdx.x; q < k * L; q += blockDim.x) sh[q] = 0;
        __syncthreads();
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        unsigned r = (unsigned)region[i], l = (unsigned)delta[i];
        if (r < (unsigned)k && l < (unsigned)L) atomicAdd(LDS ? &sh[(size_t)r * L + l] : &H[(size_t)r * L + l], 1);
    }
    if (LDS) {
        __syncthreads();
        for (int q = threadIdx.x; q < k * L; q += blockDim.x)
            if (sh[q]) atomicAdd(&H[q], sh[q]);
    }
}

__global__ void k_terms_hist_scan(int k, int L, int* __restrict__ H) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k; t += gridDim.x * blockDim.x) {
        int acc = 0;
        for (int l = 0; l < L; ++l) {
            acc += H[(size_t)t * L + l];
            H[(size_t)t * L + l] = acc;
        }
    }
}

// wtab[t][d] = H[t][min(floor(d/2), delta_max)] / d^2 for d >= 2, else 0;
// one correctly rounded FP64 division, FP32 copy rounded from it.  Padded
// ranks t >= k get zero rows.  Pivot padding repeats pivots[0].
__global__ void k_terms_wtab(int k, int kpad, int W, int delta_max, const int* __restrict__ H,
                             const int* __restrict__ pivots_in, int* __restrict__ pivots,
                             double* __restrict__ w64, float* __restrict__ w32) {
    long long total = (long long)kpad * W;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        int t = (int)(q / W), d = (int)(q % W);
        double val = 0.0;
        if (t < k && d >= 2) {
            int half = d / 2;
            if (half > delta_max) half = delta_max;
            int s = H[(size_t)t * (delta_max + 1) + half];
            val = (double)s / (double)((long long)d * (long long)d);
        }
        w64[q] = val;
        w32[q] = (float)val;
        if (d == 0) pivots[t] = pivots_in[t < k ? t : 0];
    }
}

// Tables of the FP32 sweep: wt2[t][d] = (w', w' d) rounded from FP64;
// Hf[t][l] = H[t][l] (exact in float below 2^24); invd[d] = (1/d^2, 1/d)
// for d >= 2.
__global__ void k_terms_f32_tables(int k, int kpad, int W, int L, const int* __restrict__ H,
                                   const double* __restrict__ w64, float2* __restrict__ wt2,
                                   float* __restrict__ Hf, float2* __restrict__ invd) {
    long long total = (long long)kpad * W;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        int d = (int)(q % W);
        double w = w64[q];
        wt2[q] = make_float2((float)w, (float)(w * (double)d));
    }
    long long th = (long long)kpad * L;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < th;
         q += (long long)gridDim.x * blockDim.x) {
        int t = (int)(q / L), l = (int)(q % L);
        Hf[q] = t < k ? (float)H[(size_t)t * L + l] : 0.f;
    }
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < W; d += gridDim.x * blockDim.x)
        invd[d] = d >= 2 ? make_float2((float)(1.0 / ((double)d * (double)d)), (float)(1.0 / (double)d))
                         : make_float2(0.f, 0.f);
}

// prank[i] = t for i = pivots[t], t < k; -1 elsewhere (pivots are distinct):
// a fill, then one write per pivot.
__global__ void k_terms_prank(int n, int* __restrict__ prank) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) prank[i] = -1;
}

__global__ void k_terms_prank_set(int k, const int* __restrict__ pivots, int* __restrict__ prank) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k; t += gridDim.x * blockDim.x) prank[pivots[t]] = t;
}

// den_i = deg(i) * 1 + sum over ranks t ascending of w'_it (d >= 2); summed in
// exactly that order.
__global__ void k_terms_den(int n, int k, int W, const int* __restrict__ rp, const int* __restrict__ dist,
                            const double* __restrict__ w64, double* __restrict__ den64,
                            float* __restrict__ den32) {
#pragma clang fp contract(off)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) s += 1.0;
        constexpr int U = 8;  // loads in flight; the sum keeps ascending ranks
        for (int t0 = 0; t0 < k; t0 += U) {
            int dv[U];
            double wv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) dv[j] = t0 + j < k ? dist[(size_t)(t0 + j) * n + i] : 0;
#pragma unroll
            for (int j = 0; j < U; ++j) wv[j] = dv[j] >= 2 ? w64[(size_t)(t0 + j) * W + dv[j]] : 0.0;
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (dv[j] >= 2) s += wv[j];
        }
        den64[i] = s;
        den32[i] = (float)s;
    }
}

// Packed distances: 16-byte words, word (b, i) holds dist[b*vec + j][i] for
// j < vec (uint8 when dmax <= 255, else uint16); padding ranks hold 0.
template <typename DT, int VEC>
__global__ void k_terms_pack(int n, int k, int kpad, const int* __restrict__ dist, uint4* __restrict__ out) {
    long long total = (long long)(kpad / VEC) * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        int b = (int)(q / n), i = (int)(q % n);
        union {
            uint4 v;
            DT e[VEC];
        } u;
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            int t = b * VEC + j;
            u.e[j] = t < k ? (DT)dist[(size_t)t * n + i] : (DT)0;
        }
        out[q] = u.v;
    }
}

ssm_status build_terms(const ssm_csr* g, int32_t k, const int32_t* pivots, const int32_t* dist,
                       const int32_t* delta, const int32_t* region, ssm_terms** out,
                       hipStream_t s) {
    const int n = g->n;
    int* aux = nullptr;
    ssm_status st = salloc((void**)&aux, sizeof(int) * 8);
    if (st != SSM_OK) return st;
    int h[5] = {0, 0, 0, 0, 0};
    hipError_t e = hipMemsetAsync(aux, 0, sizeof(int) * 8, s);
    const int order_mode = sweep_order_mode();
    const bool order_allowed = order_mode != 0;
    if (e == hipSuccess && order_allowed) {
        hipLaunchKernelGGL(k_order_stats, dim3(std::min(div_up(n, 256), 512)), dim3(256), 0, s, n, g->row_ptr,
                           g->col_idx, aux);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        long long total = (long long)k * n;
        // few blocks: each ends in two atomics on the same two words
        hipLaunchKernelGGL(k_terms_max, dim3((int)std::min<long long>((total + 1023) / 1024, 512)), dim3(256),
                           0, s, n, k, dist, delta, aux);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h, aux, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused
    sfree(aux);
    if (e != hipSuccess) return hip_fail(e, "terms: table extents");
    if (h[1] > 65535) return fail(SSM_E_RANGE, "distances above 65535 are not supported");

    ssm_terms* t = new ssm_terms();
    (void)hipGetDevice(&t->device);
    t->n = n;
    t->k = k;
    t->nnz = g->nnz;
    t->delta_max = h[0];
    t->dmax = h[1];
    t->dbytes = t->dmax <= 255 ? 1 : 2;
    t->vec = 16 / t->dbytes;
    t->kpad = div_up(k, t->vec) * t->vec;
    t->W = t->dmax + 1;
    const int L = t->delta_max + 1;
    const size_t kw = (size_t)t->kpad * t->W;
    t->red_len = 8192;
    // the node order pays when the labels are not local already and no hubs
    // are shared by many rows (measured on MI355X: random geometric graphs
    // gain 12-14 % per sweep; a mesh numbered along its rows and a
    // preferential-attachment graph, whose low ids are its hubs, lose)
    const double mean_deg = (double)g->nnz / (double)std::max(n, 1);
    const bool ordered = order_mode == 2 || (order_allowed && (double)h[2] <= 4.0 * std::max(mean_deg, 1.0) &&
                                             (double)h[3] < 0.5 * (double)h[4]);
    struct {
        void** p;
        size_t bytes;
    } allocs[] = {
        {(void**)&t->pivots, sizeof(int) * (size_t)t->kpad},
        {(void**)&t->H, sizeof(int) * (size_t)k * L},
        {(void**)&t->wtab64, sizeof(double) * kw},
        {(void**)&t->wtab32, sizeof(float) * kw},
        {(void**)&t->wt2, sizeof(float2) * kw},
        {(void**)&t->Hf, sizeof(float) * (size_t)t->kpad * L},
        {(void**)&t->invd, sizeof(float2) * (size_t)t->W},
        {(void**)&t->prank, sizeof(int) * (size_t)n},
        {(void**)&t->pc, sizeof(float2) * 2 * (size_t)t->kpad},
        {(void**)&t->den64, sizeof(double) * (size_t)n},
        {(void**)&t->den32, sizeof(float) * (size_t)n},
        {(void**)&t->dpk, (size_t)t->kpad * n * t->dbytes},
        {(void**)&t->xtmp, sizeof(double) * 2 * (size_t)n},
        {(void**)&t->red, sizeof(double) * (size_t)t->red_len},
        {(void**)&t->stopw, sizeof(int) * 4},
        {(void**)&t->eig, sizeof(double) * (2 * (size_t)k + 2)},
        {(void**)&t->gram, sizeof(double) * (size_t)k * k},
        {(void**)&t->eig_iters, sizeof(int)},
        // the FP32 sweep's node order (sizes 0 when off)
        {(void**)&t->perm, ordered ? sizeof(int) * (size_t)n : 0},
        {(void**)&t->inv, ordered ? sizeof(int) * (size_t)n : 0},
        {(void**)&t->prp, ordered ? sizeof(int) * ((size_t)n + 1) : 0},
        {(void**)&t->pci, ordered ? sizeof(int) * (size_t)std::max(g->nnz, 1) : 0},
        {(void**)&t->pdpk, ordered ? (size_t)t->kpad * n * t->dbytes : 0},
        {(void**)&t->pden32, ordered ? sizeof(float) * (size_t)n : 0},
        {(void**)&t->pprank, ordered ? sizeof(int) * (size_t)n : 0},
        {(void**)&t->ppiv, ordered ? sizeof(int) * (size_t)t->kpad : 0},
    };
    // one allocation, carved at 256-byte boundaries, from the scratch cache
    // (a layout pipeline builds and frees a handle of the same size each time;
    // every buffer is written before it is read)
    size_t total = 0;
    for (auto& a : allocs) total += (a.bytes + 255) / 256 * 256;
    st = salloc(&t->arena, total);
    if (st != SSM_OK) {
        ssm_terms_free(t);
        return st;
    }
    size_t off = 0;
    for (auto& a : allocs) {
        *a.p = a.bytes ? (char*)t->arena + off : nullptr;
        off += (a.bytes + 255) / 256 * 256;
    }
    int grid_n = std::min(div_up(n, 256), 8192);
    e = hipMemsetAsync(t->H, 0, sizeof(int) * (size_t)k * L, s);
    if (e == hipSuccess) e = hipMemsetAsync(t->eig_iters, 0, sizeof(int), s);
    if (e == hipSuccess) {
        if ((long long)k * L <= 8192)
            hipLaunchKernelGGL(k_terms_hist<true>, dim3(std::min(grid_n, 4 * num_cus())), dim3(256),
                               sizeof(int) * (size_t)k * L, s, n, k, L, delta, region, t->H);
        else
            hipLaunchKernelGGL(k_terms_hist<false>, dim3(grid_n), dim3(256), 0, s, n, k, L, delta, region, t->H);
        hipLaunchKernelGGL(k_terms_hist_scan, dim3(div_up(k, 256)), dim3(256), 0, s, k, L, t->H);
        hipLaunchKernelGGL(k_terms_wtab, dim3((int)std::min<long long>((kw + 255) / 256, 8192)), dim3(256), 0,
                           s, k, t->kpad, t->W, t->delta_max, t->H, pivots, t->pivots, t->wtab64, t->wtab32);
        hipLaunchKernelGGL(k_terms_f32_tables, dim3((int)std::min<long long>((kw + 255) / 256, 8192)), dim3(256),
                           0, s, k, t->kpad, t->W, L, t->H, t->wtab64, t->wt2, t->Hf, t->invd);
        hipLaunchKernelGGL(k_terms_prank, dim3(grid_n), dim3(256), 0, s, n, t->prank);
        hipLaunchKernelGGL(k_terms_prank_set, dim3(div_up(k, 256)), dim3(256), 0, s, k, pivots, t->prank);
        hipLaunchKernelGGL(k_terms_den, dim3(grid_n), dim3(256), 0, s, n, k, t->W, g->row_ptr, dist,
                           t->wtab64, t->den64, t->den32);
        long long words = (long long)(t->kpad / t->vec) * n;
        dim3 gp((int)std::min<long long>((words + 255) / 256, 16384));
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_terms_pack<uint8_t, 16>), gp, dim3(256), 0, s, n, k, t->kpad, dist,
                               (uint4*)t->dpk);
        else
            hipLaunchKernelGGL((k_terms_pack<uint16_t, 8>), gp, dim3(256), 0, s, n, k, t->kpad, dist,
                               (uint4*)t->dpk);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ssm_terms_free(t);
        return hip_fail(e, "terms: build");
    }
    // high-degree nodes (their neighbour sums get whole wavefronts)
    // the FP32 sweep's node order, then the heavy-row lists (in that order)
    st = sweep_order(g, t, delta, region, s);
    if (st != SSM_OK) {
        ssm_terms_free(t);
        return st;
    }
    *out = t;
    return SSM_OK;
}

}  // namespace ssm
