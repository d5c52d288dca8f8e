// Wavefront (64-lane) helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssm {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Rank of this lane among the set bits of `mask` below it.
__device__ __forceinline__ int mask_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Stream compaction: every active lane with `pred` gets a distinct slot from
// *tail; one atomic per wave (ballot + popcount + in-wave prefix).  Returns
// the slot, or -1 where pred is false.  Safe under divergence: the leader is
// the lowest active lane with pred set.
__device__ __forceinline__ int wave_append(bool pred, int* tail) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return -1;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(tail, __popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + mask_rank(mask) : -1;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Wave-wide sum and maximum of doubles by DPP lane moves, which stay in
// registers (a shuffle step is an LDS permute and its round trip): pairs,
// quads, half rows and rows of 16 lanes by quad permutes and mirrors, then
// the row broadcasts 15 and 31 gather the four rows into lane 63, whose
// value every lane receives.  Call with every lane of the wave active.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double old, double v) {
    const long long b = __builtin_bit_cast(long long, v), o = __builtin_bit_cast(long long, old);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane63(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0xB1, 0xf>(0.0, v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E, 0xf>(0.0, v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141, 0xf>(0.0, v);  // row_half_mirror
    v += dpp_move<0x140, 0xf>(0.0, v);  // row_mirror
    v += dpp_move<0x142, 0xa>(0.0, v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(0.0, v);  // row_bcast:31 into rows 2 and 3
    return lane63(v);
}

__device__ __forceinline__ double wave_max_dpp(double v) {
    double o;
    o = dpp_move<0xB1, 0xf>(v, v);
    v = o > v ? o : v;
    o = dpp_move<0x4E, 0xf>(v, v);
    v = o > v ? o : v;
    o = dpp_move<0x141, 0xf>(v, v);
    v = o > v ? o : v;
    o = dpp_move<0x140, 0xf>(v, v);
    v = o > v ? o : v;
    o = dpp_move<0x142, 0xa>(v, v);
    v = o > v ? o : v;
    o = dpp_move<0x143, 0xc>(v, v);
    v = o > v ? o : v;
    return lane63(v);
}

// Block-wide sum; every thread gets the result.  `scratch` holds one slot per
// wave.  Contains __syncthreads(); call from uniform control flow.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    v = wave_sum(v);
    int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    T s = 0;
    for (int q = 0; q < nw; ++q) s += scratch[q];  // fixed order: deterministic
    return s;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* scratch) {
    v = wave_max(v);
    int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    T s = scratch[0];
    for (int q = 1; q < nw; ++q) s = scratch[q] > s ? scratch[q] : s;
    return s;
}

// Calls f(i, j) for every arc (i, j) of the CSR rows i0 .. i0+63 (rows
// beyond n are empty): the wave walks the rows' arcs 64 at a time, so a
// long row costs its length / 64 passes instead of stalling one lane.  Lane
// l takes arcs e0 + l, e0 + l + 64, ... in that order, four per pass with
// their column loads in flight together.  Call with every lane of the wave
// active.
template <typename F>
__device__ __forceinline__ void wave_arcs(int n, const int* __restrict__ rp, const int* __restrict__ ci, int i0,
                                          F f) {
    constexpr int U = 4;
    const int lane = lane_id();
    const int end = rp[min(i0 + kWave, n)];
    const int a = i0 + lane < n ? rp[i0 + lane] : end;  // row start of this lane's node
    const int e0 = __shfl(a, 0);
    for (int eb = e0; eb < end; eb += U * kWave) {  // uniform
        int row[U], col[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = eb + u * kWave + lane;
            // the arc's row: the last lane whose row starts at or before e
            int lo = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1) {
                const int c = lo + step;
                if (__shfl(a, c) <= e) lo = c;
            }
            row[u] = i0 + lo;
            col[u] = e < end ? ci[e] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (eb + u * kWave + lane < end) f(row[u], col[u]);
    }
}

// Calls f(i, j) for every arc e in [a0, a1) of a CSR graph (i = the row of
// arc e, j = ci[e]), 64 arcs per pass: lane l takes arcs a0 + l, a0 + l + 64,
// ... in that order.  The row of a0 comes from a binary search over rp; a
// pass then finds its arcs' rows among the next 64 row starts (lane q holds
// the start of row r + 1 + q), so splitting [0, nnz) evenly over waves
// balances the work however long the rows are.  Call with every lane of the
// wave active.
template <typename F>
__device__ __forceinline__ void wave_arc_span(int n, const int* __restrict__ rp, const int* __restrict__ ci, int a0,
                                              int a1, F f) {
    if (a0 >= a1) return;  // uniform
    const int lane = lane_id();
    int lo = 0, hi = n;  // the last row whose start is at most a0
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rp[mid] <= a0) lo = mid;
        else hi = mid;
    }
    int r = lo;
    for (int eb = a0; eb < a1; eb += kWave) {  // uniform
        const int q = r + 1 + lane;
        const int st = q <= n ? rp[q] : 0x7fffffff;  // start of row r + 1 + lane (non-decreasing)
        const int e = eb + lane;
        int cnt = 0;  // row starts among these 64 that are at most e
#pragma unroll
        for (int step = kWave / 2; step > 0; step >>= 1) {
            const int c = cnt + step;
            if (__shfl(st, c - 1) <= e) cnt = c;
        }
        const int st_last = __shfl(st, kWave - 1);  // every lane takes part in the shuffle
        if (cnt == kWave - 1 && st_last <= e) cnt = kWave;
        int row = r + cnt;
        if (cnt == kWave && e < a1) {  // more than 64 rows begin in this pass (empty rows): search rp
            int l2 = r + kWave, h2 = n;
            while (h2 - l2 > 1) {
                const int mid = (l2 + h2) >> 1;
                if (rp[mid] <= e) l2 = mid;
                else h2 = mid;
            }
            row = l2;
        }
        if (e < a1) f(row, ci[e]);
        r = __shfl(row, min(kWave, a1 - eb) - 1);  // the row of this pass's last arc
    }
}

}  // namespace ssm
