// Localized majorization sweeps (paper Eq. 5, Algorithm 1 lines 5-8) in
// Jacobi order, and the stress of Eq. 3 and Eq. 1.
#include <float.h>
#include <math.h>
#include <stdlib.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "change.h"
#include "ssm_internal.h"
#include "sweep_f32.h"
#include "wave.h"

namespace ssm {

// ------------------------------------------------------------- reductions

// out[0] = sum of partials[0..count) in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partials, int count,
                                                      double* __restrict__ out) {
    double s = 0.0;
    for (int q = threadIdx.x; q < count; q += blockDim.x) s += partials[q];
    __shared__ double red[256 / kWave];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

void launch_sum_partials(const double* partials, int count, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, count, out);
}

// --------------------------------------------------------- FP64 sweep

// One thread per node.  Terms are summed exactly in the order stated by the
// update: neighbours at a positive distance in CSR order (w = 1, d = 1), then
// the neighbours at distance zero (each votes x_q = x_i), then pivot terms in
// ascending rank; vote(q, d) = x_q + (d (x_i - x_q)) / r, or x_q when r = 0;
// correctly rounded sqrt and division, no contraction into fused
// multiply-adds.  x_new_i = num / den_i.
template <typename DT, int VEC>
__global__ __launch_bounds__(256) void k_sweep_f64(int n, int kpad, int W, const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const double2* __restrict__ xo,
                                                   double2* __restrict__ xn, const uint4* __restrict__ dpk,
                                                   const int* __restrict__ piv,
                                                   const double* __restrict__ wt,
                                                   const double* __restrict__ den, const int* __restrict__ stop) {
#pragma clang fp contract(off)
    if (stop[0]) return;  // the sweep loop has met its stop test (uniform over the grid)
    extern __shared__ double2 sP[];
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) sP[t] = xo[piv[t]];
    __syncthreads();
    const int nwords = kpad / VEC;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double2 xv = xo[i];
        const double xi = xv.x, yi = xv.y;
        double nx = 0.0, ny = 0.0;
        int zero = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const double2 xj = xo[ci[e]];
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
            Packed<DT, VEC> u;
            u.v = dpk[(size_t)b * n + i];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const int d = (int)u.e[j];
                if (d < 2) continue;
                const int t = b * VEC + j;
                const double w = wt[(size_t)t * W + d];
                const double2 p = sP[t];
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
        const double dn = den[i];
        xn[i] = make_double2(nx / dn, ny / dn);
    }
}

// The same FP64 sweep for small graphs, where one thread per node leaves most
// of the device idle and each node's chain of square roots and divisions sets
// the time: a group of kF64Lanes lanes evaluates a node's terms in parallel
// (neighbour j by lane j mod G, pivot rank t by lane t mod G), each term's
// value (the neighbour vote, or w times the pivot vote; exactly 0 for a
// neighbour at distance zero and a pivot rank with d < 2) into LDS; then the
// group's first lane adds them in k_sweep_f64's order (neighbours in CSR
// order, x_i once per neighbour at distance zero, pivot ranks ascending).
// Adding an exact 0 changes no partial sum (a sum started at +0 never becomes
// -0), so the result is k_sweep_f64's bit for bit.  Needs degree <=
// kHeavyDegree (no heavy rows) and kpad <= kF64MaxK.
constexpr int kF64Lanes = 16;
constexpr int kF64TermsMaxN = 65536;
constexpr int kF64MaxK = 128;
constexpr int kF64Nodes = 256 / kF64Lanes;  // nodes per 256-thread block

// Element idx of a packed distance word (the little-endian DT lanes of the
// uint4), by shifts: a private array indexed at run time would live in
// scratch memory, a round trip per read.
template <typename DT>
__device__ __forceinline__ int packed_at(const uint4 v, int idx) {
    constexpr int per = 4 / (int)sizeof(DT), bits = 8 * (int)sizeof(DT);
    const int wi = idx / per;
    const unsigned w = wi == 0 ? v.x : wi == 1 ? v.y : wi == 2 ? v.z : v.w;
    return (int)((w >> ((idx % per) * bits)) & ((1u << bits) - 1u));
}

template <typename DT, int VEC>
__global__ __launch_bounds__(256) void k_sweep_f64_terms(int n, int kpad, int W, const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         const double2* __restrict__ xo,
                                                         double2* __restrict__ xn, const uint4* __restrict__ dpk,
                                                         const int* __restrict__ piv,
                                                         const double* __restrict__ wt,
                                                         const double* __restrict__ den,
                                                         const int* __restrict__ stop) {
#pragma clang fp contract(off)
    if (stop[0]) return;  // the sweep loop has met its stop test (uniform over the grid)
    extern __shared__ double2 sm[];
    const int cap = kHeavyDegree + kpad;                 // term slots per node
    double2* sP = sm;                                    // [kpad]
    double2* sT = sm + kpad;                             // [kF64Nodes][cap]
    int* sZero = (int*)(sT + (size_t)kF64Nodes * cap);  // [kF64Nodes]
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) sP[t] = xo[piv[t]];
    const int grp = threadIdx.x / kF64Lanes, lane = threadIdx.x % kF64Lanes;
    double2* T = sT + (size_t)grp * cap;
    for (int i0 = blockIdx.x * kF64Nodes; i0 < n; i0 += gridDim.x * kF64Nodes) {  // uniform over the block
        if (lane == 0) sZero[grp] = 0;
        __syncthreads();  // pivot coordinates staged; the previous nodes' terms read
        const int i = i0 + grp;
        double xi = 0.0, yi = 0.0;
        int e0 = 0, deg = 0;
        if (i < n) {
            const double2 xv = xo[i];
            xi = xv.x;
            yi = xv.y;
            e0 = rp[i];
            deg = rp[i + 1] - e0;
            for (int j = lane; j < deg; j += kF64Lanes) {
                const double2 xj = xo[ci[e0 + j]];
                double dx = xi - xj.x, dy = yi - xj.y;
                double r = sqrt(dx * dx + dy * dy);
                double2 v = make_double2(0.0, 0.0);
                if (r > 0.0)
                    v = make_double2(xj.x + dx / r, xj.y + dy / r);
                else
                    atomicAdd(&sZero[grp], 1);
                T[j] = v;
            }
            for (int t = lane; t < kpad; t += kF64Lanes) {
                const int d = packed_at<DT>(dpk[(size_t)(t / VEC) * n + i], t % VEC);
                double2 v = make_double2(0.0, 0.0);
                if (d >= 2) {
                    const double w = wt[(size_t)t * W + d];
                    const double2 p = sP[t];
                    double dx = xi - p.x, dy = yi - p.y;
                    double r = sqrt(dx * dx + dy * dy);
                    double vx = p.x, vy = p.y;
                    if (r > 0.0) {
                        vx = p.x + (double)d * dx / r;
                        vy = p.y + (double)d * dy / r;
                    }
                    v = make_double2(w * vx, w * vy);
                }
                T[kHeavyDegree + t] = v;
            }
        }
        __syncthreads();
        if (i < n && lane == 0) {
            double nx = 0.0, ny = 0.0;
            for (int j = 0; j < deg; ++j) {
                nx += T[j].x;
                ny += T[j].y;
            }
            for (int z = sZero[grp]; z > 0; --z) {
                nx += xi;
                ny += yi;
            }
            for (int t = 0; t < kpad; ++t) {
                nx += T[kHeavyDegree + t].x;
                ny += T[kHeavyDegree + t].y;
            }
            const double dn = den[i];
            xn[i] = make_double2(nx / dn, ny / dn);
        }
    }
}

// LDS bytes of k_sweep_f64_terms for kpad.
static size_t f64_terms_lds(int kpad) {
    return sizeof(double2) * ((size_t)kpad + (size_t)kF64Nodes * (kHeavyDegree + kpad)) + sizeof(int) * kF64Nodes;
}

// pc[t] = pc[kpad + t] = x[pivots[t]] for every padded rank (padding repeats
// pivots[0]; the sweeps keep only the real ranks current, the padded ones
// stay finite and carry zero weight).
__global__ void k_gather_pivots(int kpad, const int* __restrict__ piv, const float2* __restrict__ x,
                                float2* __restrict__ pc) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < kpad; t += gridDim.x * blockDim.x) {
        const float2 v = x[piv[t]];
        pc[t] = v;
        pc[kpad + t] = v;
    }
}

// Heavy list, segments and scratch of a handle (called by build_terms).
// counts[h] = segments of heavy row h, counts[nheavy] = 0 (the exclusive
// scan of the nheavy + 1 counts then ends in the total).
__global__ void k_heavy_segcount(int nheavy, const int* __restrict__ heavy, const int* __restrict__ rp,
                                 int* __restrict__ counts) {
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h <= nheavy; h += gridDim.x * blockDim.x) {
        if (h == nheavy) {
            counts[h] = 0;
            continue;
        }
        const int i = heavy[h];
        counts[h] = (rp[i + 1] - rp[i] + kHeavySeg - 1) / kHeavySeg;
    }
}

__global__ void k_heavy_segowner(int nheavy, const int* __restrict__ heavy, const int* __restrict__ seg_start,
                                 int* __restrict__ seg_owner, int2* __restrict__ seg_range) {
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < nheavy; h += gridDim.x * blockDim.x) {
        seg_range[heavy[h]] = make_int2(seg_start[h], seg_start[h + 1]);
        for (int q = seg_start[h]; q < seg_start[h + 1]; ++q) seg_owner[q] = h;
    }
}

ssm_status heavy_segments(const ssm_csr* g, ssm_terms* t, hipStream_t s) {
    ssm_status st = heavy_list(g, &t->heavy, &t->nheavy, s);
    if (st != SSM_OK) return st;
    const int nh = t->nheavy;
    st = salloc((void**)&t->seg_start, sizeof(int) * ((size_t)nh + 1));
    if (st == SSM_OK) st = salloc((void**)&t->seg_range, sizeof(int2) * (size_t)g->n);
    if (st != SSM_OK) return st;
    const int hb = std::max(1, std::min(div_up(nh + 1, 256), 1024));
    // segment counts, then their exclusive scan (the last entry is the total)
    size_t scan_bytes = 0;
    SSM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (const int*)nullptr, (int*)nullptr, nh + 1, s));
    void* scan_tmp = nullptr;
    int* counts = nullptr;
    st = salloc(&scan_tmp, std::max<size_t>(scan_bytes, 16));
    if (st == SSM_OK) st = salloc((void**)&counts, sizeof(int) * ((size_t)nh + 1));
    if (st != SSM_OK) {
        if (scan_tmp) sfree(scan_tmp);
        return st;
    }
    hipLaunchKernelGGL(k_heavy_segcount, dim3(hb), dim3(256), 0, s, nh, t->heavy, g->row_ptr, counts);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, counts, t->seg_start, nh + 1, s);
    int nseg = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&nseg, t->seg_start + nh, sizeof(int), hipMemcpyDeviceToHost, s);
    const hipError_t es = hipStreamSynchronize(s);
    sfree(counts);
    sfree(scan_tmp);
    SSM_HIP(e);
    SSM_HIP(es);
    t->nseg = nseg;
    st = salloc((void**)&t->seg_owner, sizeof(int) * (size_t)std::max(nseg, 1));
    if (st == SSM_OK) st = salloc((void**)&t->seg_sum, sizeof(float2) * (size_t)std::max(nseg, 1));
    if (st != SSM_OK) return st;
    hipLaunchKernelGGL(k_heavy_segowner, dim3(hb), dim3(256), 0, s, nh, t->heavy, t->seg_start, t->seg_owner,
                       t->seg_range);
    SSM_HIP(hipGetLastError());
    SSM_HIP(hipStreamSynchronize(s));
    return SSM_OK;
}

// ------------------------------------------------ FP32 sweep node order

int sweep_order_mode() {  // variant sweep_perm: -1 = the caller's order, 2 = always reorder
    const int m = variant("sweep_perm");
    return m == -1 ? 0 : m == 2 ? 2 : 1;
}

__global__ void k_order_keys(int n, const int* __restrict__ delta, const int* __restrict__ region,
                             unsigned long long* __restrict__ key, int* __restrict__ val) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        key[i] = ((unsigned long long)(unsigned)region[i] << 32) | (unsigned)delta[i];
        val[i] = i;
    }
}

// Per new row r (node perm[r]): inv, row length, denominator, pivot rank.
__global__ void k_order_rows(int n, const int* __restrict__ perm, const int* __restrict__ rp,
                             const float* __restrict__ den32, const int* __restrict__ prank, int* __restrict__ inv,
                             int* __restrict__ deg, float* __restrict__ pden, int* __restrict__ pprank) {
    if (blockIdx.x == 0 && threadIdx.x == 0) deg[n] = 0;  // the scan's last entry
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int o = perm[r];
        inv[o] = r;
        deg[r] = rp[o + 1] - rp[o];
        pden[r] = den32[o];
        pprank[r] = prank[o];
    }
}

// Renumbered rows: row r is node perm[r]'s row, its neighbours' new ids in
// the same order.
__global__ void k_order_csr(int n, const int* __restrict__ perm, const int* __restrict__ inv,
                            const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ prp,
                            int* __restrict__ pci) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int o = perm[r], a = rp[o], d = rp[o + 1] - a, b = prp[r];
        for (int j = 0; j < d; ++j) pci[b + j] = inv[ci[a + j]];
    }
}

// Packed distances in the new order: word b of node perm[r] (already packed
// by build_terms) moves to word b of r, one 16-byte gather per word.
__global__ void k_order_pack(int n, int nwords, const int* __restrict__ perm, const uint4* __restrict__ dpk,
                             uint4* __restrict__ out) {
    const long long total = (long long)nwords * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int b = (int)(q / n), r = (int)(q % n);
        out[q] = dpk[(size_t)b * n + perm[r]];
    }
}

__global__ void k_order_piv(int kpad, const int* __restrict__ piv, const int* __restrict__ inv, int* __restrict__ ppiv) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < kpad; t += gridDim.x * blockDim.x) ppiv[t] = inv[piv[t]];
}

__global__ void k_perm_gather(int n, const int* __restrict__ perm, const float2* __restrict__ x, float2* __restrict__ y) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) y[r] = x[perm[r]];
}

__global__ void k_perm_scatter(int n, const int* __restrict__ perm, const float2* __restrict__ y, float2* __restrict__ x) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) x[perm[r]] = y[r];
}

ssm_status sweep_order(const ssm_csr* g, ssm_terms* t, const int32_t* delta,
                       const int32_t* region, hipStream_t s) {
    if (!t->perm) return heavy_segments(g, t, s);
    const int n = t->n;
    const int gb = std::min(div_up(n, 256), 8192);
    // scratch: keys (2 n u64), values (n ints), row lengths (n + 1 ints), sort and scan space
    size_t sort_bytes = 0, scan_bytes = 0;
    SSM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (unsigned long long*)nullptr,
                                               (unsigned long long*)nullptr, (int*)nullptr, (int*)nullptr, n, 0,
                                               64, s));
    SSM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int*)nullptr, (int*)nullptr, n + 1, s));
    const size_t tmp_bytes = std::max(sort_bytes, scan_bytes);
    const size_t bytes = sizeof(unsigned long long) * 2 * (size_t)n + sizeof(int) * (2 * (size_t)n + 1) + tmp_bytes + 512;
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, bytes);
    if (st != SSM_OK) return st;
    unsigned long long* kin = (unsigned long long*)ws;
    unsigned long long* kout = kin + n;
    int* vin = (int*)(kout + n);
    int* deg = vin + n;
    void* tmp = (void*)(((uintptr_t)(deg + n + 1) + 255) & ~(uintptr_t)255);
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_order_keys, dim3(gb), dim3(256), 0, s, n, delta, region, kin, vin);
    size_t tb = sort_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, vin, t->perm, n, 0, 64, s);  // stable: ids ascend
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_order_rows, dim3(gb), dim3(256), 0, s, n, t->perm, g->row_ptr, t->den32, t->prank,
                           t->inv, deg, t->pden32, t->pprank);
        size_t sb = scan_bytes;
        e = hipcub::DeviceScan::ExclusiveSum(tmp, sb, deg, t->prp, n + 1, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_order_csr, dim3(gb), dim3(256), 0, s, n, t->perm, t->inv, g->row_ptr, g->col_idx,
                           t->prp, t->pci);
        const long long words = (long long)(t->kpad / t->vec) * n;
        const dim3 gp((int)std::min<long long>((words + 255) / 256, 16384));
        hipLaunchKernelGGL(k_order_pack, gp, dim3(256), 0, s, n, t->kpad / t->vec, t->perm, (const uint4*)t->dpk,
                           (uint4*)t->pdpk);
        hipLaunchKernelGGL(k_order_piv, dim3(div_up(t->kpad, 256)), dim3(256), 0, s, t->kpad, t->pivots, t->inv,
                           t->ppiv);
        e = hipGetLastError();
    }
    const hipError_t e2 = hipStreamSynchronize(s);  // idle before the scratch is reused
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "terms: sweep order");
    if (e2 != hipSuccess) return hip_fail(e2, "terms: sweep order");
    const ssm_csr gp = {n, t->nnz, t->prp, t->pci};
    return heavy_segments(&gp, t, s);
}

// ----------------------------------------------------------- stress

template <typename T2>
__device__ __forceinline__ double2 as_d2(const T2 v) {
    return make_double2((double)v.x, (double)v.y);
}

// Per-block partials of the sparse stress s'(x), Eq. 3, in FP64.
template <typename T2, typename DT, int VEC>
__global__ __launch_bounds__(256) void k_stress(int n, int kpad, int W, const int* __restrict__ rp,
                                                const int* __restrict__ ci, const T2* __restrict__ x,
                                                const uint4* __restrict__ dpk, const int* __restrict__ piv,
                                                const double* __restrict__ wt,
                                                double* __restrict__ partials) {
    extern __shared__ double2 sQ[];
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) sQ[t] = as_d2(x[piv[t]]);
    __syncthreads();
    const int nwords = kpad / VEC;
    double acc = 0.0;
    // the edge terms (i < j): every wave an equal share of the arcs; then
    // the pivot terms: waves walk chunks of 64 nodes
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nwaves = gridDim.x * blockDim.x / kWave;
    const long long nnz = rp[n];
    wave_arc_span(n, rp, ci, (int)(nnz * wave / nwaves), (int)(nnz * (wave + 1) / nwaves), [&](int i, int j) {
        if (j <= i) return;
        const double2 xi = as_d2(x[i]), xj = as_d2(x[j]);
        double dx = xi.x - xj.x, dy = xi.y - xj.y;
        double r = sqrt(dx * dx + dy * dy);
        acc += (r - 1.0) * (r - 1.0);
    });
    for (int i0 = wave * kWave; i0 < n; i0 += nwaves * kWave) {
        const int i = i0 + lane_id();
        if (i >= n) continue;
        const double2 xi = as_d2(x[i]);
        for (int b = 0; b < nwords; ++b) {
            Packed<DT, VEC> u;
            u.v = dpk[(size_t)b * n + i];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const int d = (int)u.e[j];
                if (d < 2) continue;
                const int t = b * VEC + j;
                const double2 p = sQ[t];
                double dx = xi.x - p.x, dy = xi.y - p.y;
                double r = sqrt(dx * dx + dy * dy);
                acc += wt[(size_t)t * W + d] * (r - d) * (r - d);
            }
        }
    }
    __shared__ double red[256 / kWave];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Algorithm 1's stop test after a sweep xo -> xn (change.h): per-block
// partials of the twelve moments, relative to o = xo[0].
template <typename T2>
__global__ __launch_bounds__(256) void k_rigid_moments(int n, const T2* __restrict__ xo, const T2* __restrict__ xn,
                                                       const int* __restrict__ stop, double* __restrict__ partials) {
    if (stop[0]) return;
    const double2 o = to_d2(xo[0]);
    double m[kMoments];
#pragma unroll
    for (int j = 0; j < kMoments; ++j) m[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        moments_add(m, o, to_d2(xo[i]), to_d2(xn[i]));
    __shared__ double red[(256 / kWave) * kMoments];
    const double v = block_moments(m, red);
    if (threadIdx.x < kMoments) partials[(size_t)blockIdx.x * kMoments + threadIdx.x] = v;
}

// One block: sums the partials in a fixed order; after sweep `it` (0-based)
// of the loop, a change <= tol sets the stop flag and records it + 1 sweeps.
// stopw = {flag, sweeps run}.
__global__ __launch_bounds__(256) void k_rigid_decide(int nblocks, const double* __restrict__ partials, int n,
                                                      double tol, int it, int* __restrict__ stopw,
                                                      double* __restrict__ last_change) {
    if (stopw[0]) return;
    __shared__ double red[(256 / kWave) * kMoments];
    __shared__ double s_m[kMoments];
    double m[kMoments];
#pragma unroll
    for (int j = 0; j < kMoments; ++j) {
        double v = 0.0;
        for (int q = threadIdx.x; q < nblocks; q += blockDim.x) v += partials[(size_t)q * kMoments + j];
        m[j] = v;
    }
    const double v = block_moments(m, red);
    if (threadIdx.x < kMoments) s_m[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < kMoments; ++j) m[j] = s_m[j];
        const double c = rigid_change(m, n);
        last_change[0] = c;
        if (c <= tol) {
            stopw[0] = 1;
            stopw[1] = it + 1;
        }
    }
}

// stopw = {0 (not stopped), iters (sweeps run unless the test fires)}.
__global__ void k_stop_init(int* stopw, int iters) {
    if (threadIdx.x == 0) {
        stopw[0] = 0;
        stopw[1] = iters;
    }
}

// After a loop with a stop test: the result lies in buffer (sweeps run) & 1;
// bring it to buffer 0.
template <typename T2>
__global__ void k_stop_result(int n, const int* __restrict__ stopw, T2* __restrict__ b0, const T2* __restrict__ b1) {
    if (!(stopw[1] & 1)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b0[i] = b1[i];
}

// -------------------------------------------------------------- driver

constexpr int kStopBlocks = 512;  // blocks of the stop test's moments (partials fit the handle's scratch)

struct SweepPlan {
    int grid = 1, block = 256, split = 4, cpb = 4, mode = kTableGlobal;
    size_t lds = 0;
    bool nt = false;         // non-temporal distance loads
    bool f64_terms = false;  // FP64: k_sweep_f64_terms (small graphs)
};

// Distance streams above half the MALL (256 MB on MI355X) are read with
// non-temporal loads (sweep_f32.h).
constexpr size_t kStreamNtBytes = 128u << 20;

template <typename DT, int VEC, int SPLIT, int CPB, int MODE>
static void launch_f32(const SweepPlan& pl, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                       const float2* xo, float2* xn, const float2* pc, float2* pc_next) {
    if (pl.lds > 64 * 1024)  // above the default dynamic LDS limit
        (void)hipFuncSetAttribute((const void*)k_sweep_f32<DT, VEC, SPLIT, CPB, MODE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
    hipLaunchKernelGGL((k_sweep_f32<DT, VEC, SPLIT, CPB, MODE>), dim3(pl.grid), dim3(64 * SPLIT * CPB), pl.lds, s,
                       t->n, t->kpad, t->W, t->delta_max + 1, g->row_ptr, g->col_idx, xo, xn, (const uint4*)t->dpk,
                       pc, pc_next, t->prank, t->wt2, t->Hf, t->invd, t->den32, t->seg_range, t->seg_sum, t->stopw,
                       pl.nt);
}

template <typename DT, int VEC, int SPLIT, int CPB>
static void dispatch_mode(const SweepPlan& pl, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                          const float2* xo, float2* xn, const float2* pc, float2* pc_next) {
    switch (pl.mode) {
        case kTableLds: launch_f32<DT, VEC, SPLIT, CPB, kTableLds>(pl, s, g, t, xo, xn, pc, pc_next); break;
        case kHistLds: launch_f32<DT, VEC, SPLIT, CPB, kHistLds>(pl, s, g, t, xo, xn, pc, pc_next); break;
        default: launch_f32<DT, VEC, SPLIT, CPB, kTableGlobal>(pl, s, g, t, xo, xn, pc, pc_next); break;
    }
}

// Blocks of 4 waves (small LDS tables) or 16 waves (one large table per CU):
// SPLIT waves per 64-node chunk.
template <typename DT, int VEC>
static void dispatch_split(const SweepPlan& pl, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                           const float2* xo, float2* xn, const float2* pc, float2* pc_next) {
    const bool big = pl.block == 1024;
    switch (pl.split) {
        case 1:
            if (big) dispatch_mode<DT, VEC, 1, 16>(pl, s, g, t, xo, xn, pc, pc_next);
            else dispatch_mode<DT, VEC, 1, 4>(pl, s, g, t, xo, xn, pc, pc_next);
            break;
        case 2:
            if (big) dispatch_mode<DT, VEC, 2, 8>(pl, s, g, t, xo, xn, pc, pc_next);
            else dispatch_mode<DT, VEC, 2, 2>(pl, s, g, t, xo, xn, pc, pc_next);
            break;
        default:
            if (big) dispatch_mode<DT, VEC, 4, 4>(pl, s, g, t, xo, xn, pc, pc_next);
            else dispatch_mode<DT, VEC, 4, 1>(pl, s, g, t, xo, xn, pc, pc_next);
            break;
    }
}

// One sweep xo -> xn.  FP32: pc holds the pivot coordinates of xo; the sweep
// writes those of xn into pc_next.
static void sweep_once(const SweepPlan& pl, ssm_prec p, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                       const void* xo, void* xn, const float2* pc = nullptr, float2* pc_next = nullptr) {
    if (p == SSM_FP64 && pl.f64_terms) {
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_sweep_f64_terms<uint8_t, 16>), dim3(pl.grid), dim3(256), pl.lds, s, t->n, t->kpad,
                               t->W, g->row_ptr, g->col_idx, (const double2*)xo, (double2*)xn,
                               (const uint4*)t->dpk, t->pivots, t->wtab64, t->den64, t->stopw);
        else
            hipLaunchKernelGGL((k_sweep_f64_terms<uint16_t, 8>), dim3(pl.grid), dim3(256), pl.lds, s, t->n, t->kpad,
                               t->W, g->row_ptr, g->col_idx, (const double2*)xo, (double2*)xn,
                               (const uint4*)t->dpk, t->pivots, t->wtab64, t->den64, t->stopw);
        return;
    }
    if (p == SSM_FP64) {
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_sweep_f64<uint8_t, 16>), dim3(pl.grid), dim3(pl.block), pl.lds, s, t->n, t->kpad,
                               t->W, g->row_ptr, g->col_idx, (const double2*)xo, (double2*)xn,
                               (const uint4*)t->dpk, t->pivots, t->wtab64, t->den64, t->stopw);
        else
            hipLaunchKernelGGL((k_sweep_f64<uint16_t, 8>), dim3(pl.grid), dim3(pl.block), pl.lds, s, t->n, t->kpad,
                               t->W, g->row_ptr, g->col_idx, (const double2*)xo, (double2*)xn,
                               (const uint4*)t->dpk, t->pivots, t->wtab64, t->den64, t->stopw);
        return;
    }
    if (t->nseg > 0)
        hipLaunchKernelGGL(k_heavy_edges, dim3(std::min(div_up(t->nseg, 4), 4096)), dim3(256), 0, s, t->nseg,
                           t->heavy, t->seg_start, t->seg_owner, g->row_ptr, g->col_idx, (const float2*)xo,
                           t->seg_sum, t->stopw);
    if (t->dbytes == 1)
        dispatch_split<uint8_t, 16>(pl, s, g, t, (const float2*)xo, (float2*)xn, pc, pc_next);
    else
        dispatch_split<uint16_t, 8>(pl, s, g, t, (const float2*)xo, (float2*)xn, pc, pc_next);
}

constexpr size_t kSweepLdsMax = 150 * 1024;  // LDS of one FP32 sweep block (160 KB per CU)

// The FP32 sweep's weight form and its LDS bytes besides the partials: the
// whole (w', w' d) table when it fits, else the histograms, else the table
// in global memory (the form changes the arithmetic, so it follows from the
// table sizes alone).
static int sweep_mode(const ssm_terms* t, size_t* tab_bytes) {
    const size_t table = sizeof(float2) * (size_t)t->kpad * t->W;
    const size_t hist = sizeof(float2) * (size_t)(t->W + 1) / 2 * 2 + sizeof(float) * (size_t)t->kpad * (t->delta_max + 1);
    const size_t parts = sizeof(float2) * (2 * 16 * 2 * 64 + (size_t)t->kpad);  // partials of the largest block, pivots
    int mode = table + parts <= kSweepLdsMax ? kTableLds : hist + parts <= kSweepLdsMax ? kHistLds : kTableGlobal;
    if (const int f = variant("sweep_mode")) {  // override: 2 = global table, 1 = LDS histograms (if they fit)
        if (f == kTableGlobal || (f == kHistLds && hist + parts <= kSweepLdsMax)) mode = f;
    }
    *tab_bytes = mode == kTableLds ? table : mode == kHistLds ? hist : 0;
    return mode;
}

// An FP32 launch shape: `split` waves per 64-node chunk, `waves` per block,
// at most `bpc` blocks per CU (fewer when their LDS does not fit).
static SweepPlan shape_f32(const ssm_terms* t, int mode, size_t tab, int split, int waves, int bpc) {
    SweepPlan pl;
    pl.mode = mode;
    pl.block = 64 * waves;
    pl.split = split;
    pl.cpb = waves / split;
    pl.lds = sizeof(float2) * (size_t)t->kpad + tab + (split > 1 ? sizeof(float2) * 2 * waves * (4 / split) * 64 : 0);
    const int fit = std::max(1, (int)((160 * 1024) / std::max<size_t>(pl.lds, 1)));
    const long long groups = div_up(div_up(t->n, 64), pl.cpb);
    pl.grid = (int)std::max<long long>(1, std::min(groups, (long long)num_cus() * std::min(bpc, fit)));
    pl.nt = (size_t)t->n * t->kpad * t->dbytes > kStreamNtBytes;
    return pl;
}

// The rule shape: a large table is staged once per CU by a 16-wave block, a
// small one by 4-wave blocks (finer load balance); two waves per chunk for
// 4-wave blocks, one for 16-wave blocks; as many blocks per CU as fit, up to
// four (two 16-wave blocks).  Variants override each choice.
static SweepPlan plan_sweep(const ssm_terms* t, ssm_prec p) {
    if (p == SSM_FP64) {
        SweepPlan pl;
        pl.block = 256;
        // graphs up to kF64TermsMaxN nodes without heavy rows: a lane group
        // per node (variant sweep_f64_terms -1: a thread per node)
        pl.f64_terms = t->n <= kF64TermsMaxN && t->nheavy == 0 && t->kpad <= kF64MaxK &&
                       variant("sweep_f64_terms") != -1;
        if (pl.f64_terms) {
            pl.lds = f64_terms_lds(t->kpad);
            pl.grid = std::max(1, div_up(t->n, kF64Nodes));
            return pl;
        }
        pl.lds = sizeof(double) * 2 * (size_t)t->kpad;
        pl.grid = std::max(1, std::min(div_up(t->n, pl.block), num_cus() * 8));
        return pl;
    }
    const int nwords = t->kpad / t->vec;
    size_t tab = 0;
    const int mode = sweep_mode(t, &tab);
    int waves = tab > 40 * 1024 ? 16 : 4;
    if (const int v = variant("sweep_waves")) {
        if (v == 4 || v == 16) waves = v;
    }
    int split = std::min(waves == 16 ? 1 : 2, nwords);
    if (const int f = variant("sweep_split")) {
        if ((f == 1 || f == 2 || f == 4) && f <= nwords) split = f;
    }
    int bpc = waves == 16 ? 2 : 4;
    if (const int v = variant("sweep_blocks_per_cu")) bpc = std::max(1, v);
    return shape_f32(t, mode, tab, split, waves, bpc);
}

// ---------------------------------------------------------- autotuner
//
// The FP32 sweep's result does not depend on its launch shape (split, block
// shape, grid: see k_sweep_f32), so the first FP32 sweep loop of at least
// kTuneMinIters sweeps on a graph shape times every candidate shape for a
// few sweeps on scratch copies of the layout and keeps the fastest, per
// device and (n, arcs, padded k, table extents, distance width, node
// order).  Forced variants skip the tuning.
constexpr int kTuneMinIters = 24;

struct PlanKey {
    int dev, n, nnz, kpad, W, L, dbytes, ordered, mode;
    bool operator<(const PlanKey& o) const {
        return std::tie(dev, n, nnz, kpad, W, L, dbytes, ordered, mode) <
               std::tie(o.dev, o.n, o.nnz, o.kpad, o.W, o.L, o.dbytes, o.ordered, o.mode);
    }
};
static std::mutex g_plan_mu;
static std::map<PlanKey, SweepPlan> g_plans;

// Any forced sweep variant (the weight form included) turns the tuning off
// and leaves the cache alone.
static bool sweep_shape_forced() {
    return variant("sweep_split") || variant("sweep_blocks_per_cu") || variant("sweep_waves") ||
           variant("sweep_mode") || variant("sweep_tune") == -1;
}

// Times `reps` sweeps of plan pl on scratch buffers ya, yb (ya holds a copy
// of the layout); 0 on error.
static float time_plan(const SweepPlan& pl, hipStream_t s, const ssm_csr* g, ssm_terms* t, float2* ya, float2* yb,
                       hipEvent_t e0, hipEvent_t e1, int reps) {
    float2* pcb[2] = {t->pc, t->pc + t->kpad};
    hipLaunchKernelGGL(k_stop_init, dim3(1), dim3(64), 0, s, t->stopw, 0);
    hipLaunchKernelGGL(k_gather_pivots, dim3(div_up(t->kpad, 256)), dim3(256), 0, s, t->kpad, t->pivots,
                       (const float2*)ya, pcb[0]);
    sweep_once(pl, SSM_FP32, s, g, t, ya, yb, pcb[0], pcb[1]);  // warm
    float2* buf[2] = {yb, ya};
    if (hipEventRecord(e0, s) != hipSuccess) return 0.f;
    for (int r = 0; r < reps; ++r)
        sweep_once(pl, SSM_FP32, s, g, t, buf[r & 1], buf[(r + 1) & 1], pcb[(r + 1) & 1], pcb[r & 1]);
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 0.f;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 0.f;
    return ms;
}

static SweepPlan tuned_plan(const ssm_csr* g, ssm_terms* t, const void* x, int iters, hipStream_t s) {
    SweepPlan rule = plan_sweep(t, SSM_FP32);
    if (iters < kTuneMinIters || sweep_shape_forced()) return rule;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return rule;
    PlanKey key{t->device, t->n, t->nnz, t->kpad, t->W, t->delta_max + 1, t->dbytes, t->perm != nullptr, rule.mode};
    {
        std::lock_guard<std::mutex> lock(g_plan_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) return it->second;
    }
    const int nwords = t->kpad / t->vec;
    size_t tab = 0;
    const int mode = sweep_mode(t, &tab);
    std::vector<SweepPlan> cand;
    for (int waves : {4, 16}) {
        if (tab > 40 * 1024 && waves == 4) continue;  // a large table is staged once per CU
        for (int split : {1, 2, 4}) {
            if (split > nwords) continue;
            for (int bpc : {1, 2, 3, 4, 6, 8}) {
                if (waves == 16 && bpc > 2) continue;
                cand.push_back(shape_f32(t, mode, tab, split, waves, bpc));
            }
        }
    }
    float2* y = nullptr;
    if (salloc((void**)&y, sizeof(float2) * 2 * (size_t)t->n) != SSM_OK) return rule;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SweepPlan best = rule;
    float best_ms = 0.f;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
              hipMemcpyAsync(y, x, sizeof(float2) * (size_t)t->n, hipMemcpyDeviceToDevice, s) == hipSuccess;
    for (size_t c = 0; ok && c < cand.size(); ++c) {
        const float ms = time_plan(cand[c], s, g, t, y, y + t->n, e0, e1, 3);
        if (ms <= 0.f) {
            ok = false;
            break;
        }
        if (best_ms == 0.f || ms < best_ms) {
            best_ms = ms;
            best = cand[c];
        }
    }
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    sfree(y);
    (void)hipGetLastError();
    if (!ok) return rule;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plans[key] = best;
    return best;
}

// The sweep loop over buffers bufs[0] (in/out) and bufs[1]; the result ends
// in bufs[0].  With tol > 0, Algorithm 1's stop test runs on the device after
// every sweep (k_rigid_moments, k_rigid_decide); once it fires, the later
// sweeps of the loop return at once, and the buffer holding the result is
// chosen on the device.  Nothing waits on the host unless the sweep count is
// asked for.
static ssm_status sweep_loop(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* const (&bufs)[2], int32_t iters,
                             double tol, int32_t* iters_done_host, hipStream_t s) {
    const SweepPlan pl = p == SSM_FP32 ? tuned_plan(g, t, bufs[0], iters, s) : plan_sweep(t, p);
    const size_t xbytes = (p == SSM_FP64 ? sizeof(double) : sizeof(float)) * 2 * (size_t)t->n;
    void* const x = bufs[0];
    const int mblocks = std::min(div_up(t->n, 256), kStopBlocks);
    double* parts = t->red;
    float2* pcb[2] = {t->pc, t->pc + t->kpad};
    hipLaunchKernelGGL(k_stop_init, dim3(1), dim3(64), 0, s, t->stopw, iters);
    if (p == SSM_FP32 && iters > 0)
        hipLaunchKernelGGL(k_gather_pivots, dim3(div_up(t->kpad, 256)), dim3(256), 0, s, t->kpad, t->pivots,
                           (const float2*)x, pcb[0]);
    for (int it = 0; it < iters; ++it) {
        const int cur = it & 1;
        sweep_once(pl, p, s, g, t, bufs[cur], bufs[cur ^ 1], pcb[cur], pcb[cur ^ 1]);
        if (tol > 0.0) {
            if (p == SSM_FP64)
                hipLaunchKernelGGL(k_rigid_moments<double2>, dim3(mblocks), dim3(256), 0, s, t->n,
                                   (const double2*)bufs[cur], (const double2*)bufs[cur ^ 1], t->stopw, parts);
            else
                hipLaunchKernelGGL(k_rigid_moments<float2>, dim3(mblocks), dim3(256), 0, s, t->n,
                                   (const float2*)bufs[cur], (const float2*)bufs[cur ^ 1], t->stopw, parts);
            hipLaunchKernelGGL(k_rigid_decide, dim3(1), dim3(256), 0, s, mblocks, parts, t->n, tol, it, t->stopw,
                               parts + (size_t)kStopBlocks * kMoments);
        }
    }
    SSM_HIP(hipGetLastError());
    if (tol > 0.0) {
        const int gb = std::min(div_up(t->n, 256), 4096);
        if (p == SSM_FP64)
            hipLaunchKernelGGL(k_stop_result<double2>, dim3(gb), dim3(256), 0, s, t->n, t->stopw, (double2*)x,
                               (const double2*)bufs[1]);
        else
            hipLaunchKernelGGL(k_stop_result<float2>, dim3(gb), dim3(256), 0, s, t->n, t->stopw, (float2*)x,
                               (const float2*)bufs[1]);
        SSM_HIP(hipGetLastError());
    } else if (iters & 1) {
        SSM_HIP(hipMemcpyAsync(x, bufs[1], xbytes, hipMemcpyDeviceToDevice, s));
    }
    if (iters_done_host) {
        int32_t h[2] = {0, 0};
        SSM_HIP(hipMemcpyAsync(h, t->stopw, sizeof h, hipMemcpyDeviceToHost, s));
        SSM_HIP(hipStreamSynchronize(s));
        *iters_done_host = h[1];
    }
    return SSM_OK;
}

ssm_status majorize(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x, int32_t iters, double tol,
                    int32_t* iters_done_host, hipStream_t s) {
    if (p != SSM_FP32 || !t->perm || iters <= 0) {
        void* const bufs[2] = {x, t->xtmp};
        return sweep_loop(g, t, p, bufs, iters, tol, iters_done_host, s);
    }
    // FP32 in the sweep order: the renumbered graph and per-node data, the
    // coordinates gathered into the two halves of xtmp and scattered back
    const int n = t->n;
    const ssm_csr gp = {n, t->nnz, t->prp, t->pci};
    ssm_terms tv = *t;
    tv.dpk = t->pdpk;
    tv.den32 = t->pden32;
    tv.prank = t->pprank;
    tv.pivots = t->ppiv;
    float2* xa = (float2*)t->xtmp;
    float2* xb = xa + n;
    const int gb = std::min(div_up(n, 256), 8192);
    hipLaunchKernelGGL(k_perm_gather, dim3(gb), dim3(256), 0, s, n, t->perm, (const float2*)x, xa);
    void* const bufs[2] = {xa, xb};
    ssm_status st = sweep_loop(&gp, &tv, p, bufs, iters, tol, iters_done_host, s);
    if (st != SSM_OK) return st;
    hipLaunchKernelGGL(k_perm_scatter, dim3(gb), dim3(256), 0, s, n, t->perm, (const float2*)xa, (float2*)x);
    SSM_HIP(hipGetLastError());
    return SSM_OK;
}

__global__ void k_round_layout(int n, const double2* __restrict__ a, float2* __restrict__ b) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double2 v = a[i];
        b[i] = make_float2((float)v.x, (float)v.y);
    }
}

ssm_status majorize_mixed(const ssm_csr* g, ssm_terms* t, double* x64, float* x32, int32_t iters, int32_t warm,
                          hipStream_t s) {
    const int first = std::min(iters, warm);
    ssm_status st = majorize(g, t, SSM_FP64, x64, first, 0.0, nullptr, s);
    if (st != SSM_OK) return st;
    hipLaunchKernelGGL(k_round_layout, dim3(std::min(div_up(t->n, 256), 4096)), dim3(256), 0, s, t->n,
                       (const double2*)x64, (float2*)x32);
    SSM_HIP(hipGetLastError());
    if (iters > first) return majorize(g, t, SSM_FP32, x32, iters - first, 0.0, nullptr, s);
    return SSM_OK;
}

ssm_status stress_sparse(const ssm_csr* g, ssm_terms* t, ssm_prec p, const void* x, double* out_host,
                         hipStream_t s) {
    const int blocks = std::min(div_up(t->n, 256), std::min(2048, t->red_len - 8));
    const size_t lds = sizeof(double) * 2 * (size_t)t->kpad;
    const uint4* dpk = (const uint4*)t->dpk;
    if (p == SSM_FP64) {
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_stress<double2, uint8_t, 16>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const double2*)x, dpk, t->pivots, t->wtab64, t->red);
        else
            hipLaunchKernelGGL((k_stress<double2, uint16_t, 8>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const double2*)x, dpk, t->pivots, t->wtab64, t->red);
    } else {
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_stress<float2, uint8_t, 16>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const float2*)x, dpk, t->pivots, t->wtab64, t->red);
        else
            hipLaunchKernelGGL((k_stress<float2, uint16_t, 8>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const float2*)x, dpk, t->pivots, t->wtab64, t->red);
    }
    launch_sum_partials(t->red, blocks, t->red + blocks, s);
    SSM_HIP(hipGetLastError());
    SSM_HIP(hipMemcpyAsync(out_host, t->red + blocks, sizeof(double), hipMemcpyDeviceToHost, s));
    SSM_HIP(hipStreamSynchronize(s));
    return SSM_OK;
}

// ------------------------------------------------------ full stress (Eq. 1)

// Sources s0 .. s0+nb-1 (BFS rows D): partials of sum over j > s of
// (r - d)^2 / d^2.
template <typename T2>
__global__ __launch_bounds__(256) void k_stress_full(int n, int s0, int nb, const int* __restrict__ D,
                                                     const T2* __restrict__ x, double* __restrict__ partials) {
    double acc = 0.0;
    long long total = (long long)nb * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        int r = (int)(q / n), j = (int)(q % n);
        int src = s0 + r;
        if (j <= src) continue;
        double d = (double)D[q];
        double2 a = as_d2(x[src]), b = as_d2(x[j]);
        double dx = a.x - b.x, dy = a.y - b.y;
        double dist = sqrt(dx * dx + dy * dy);
        acc += (dist - d) * (dist - d) / (d * d);
    }
    __shared__ double red[256 / kWave];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] += acc;
}

__global__ void k_iota(int* p, int s0, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = s0 + i;
}

ssm_status stress_full(const ssm_csr* g, ssm_prec p, const void* x, double* out_host, hipStream_t s) {
    const int n = g->n;
    const int nb = std::max(1, std::min(n, (1 << 26) / n));  // rows per batch (<= 256 MiB of distances)
    const int blocks = 1024;
    int* D = nullptr;
    int* src = nullptr;
    double* part = nullptr;
    ssm_status st = salloc((void**)&D, sizeof(int) * (size_t)nb * n);
    if (st == SSM_OK) st = salloc((void**)&src, sizeof(int) * (size_t)nb);
    if (st == SSM_OK) st = salloc((void**)&part, sizeof(double) * (blocks + 1));
    if (st != SSM_OK) {  // nothing queued yet
        sfree(D);
        sfree(src);
        return st;
    }
    hipError_t e = hipMemsetAsync(part, 0, sizeof(double) * (blocks + 1), s);
    for (int s0 = 0; s0 < n && e == hipSuccess && st == SSM_OK; s0 += nb) {
        int cnt = std::min(nb, n - s0);
        hipLaunchKernelGGL(k_iota, dim3(div_up(cnt, 256)), dim3(256), 0, s, src, s0, cnt);
        int32_t dm = 0;
        st = mssp(g, cnt, src, D, &dm, s);
        if (st != SSM_OK) break;
        if (p == SSM_FP64)
            hipLaunchKernelGGL(k_stress_full<double2>, dim3(blocks), dim3(256), 0, s, n, s0, cnt, D,
                               (const double2*)x, part);
        else
            hipLaunchKernelGGL(k_stress_full<float2>, dim3(blocks), dim3(256), 0, s, n, s0, cnt, D,
                               (const float2*)x, part);
        e = hipGetLastError();
    }
    if (st == SSM_OK && e == hipSuccess) {
        launch_sum_partials(part, blocks, part + blocks, s);
        e = hipMemcpyAsync(out_host, part + blocks, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused (also after an error)
    sfree(D);
    sfree(src);
    sfree(part);
    if (st != SSM_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "full stress");
    return SSM_OK;
}

}  // namespace ssm
